// opo.hip -- host side of the C ABI declared in include/opo.h: validation,
// planning (four-step split, tile shapes, FP64 tables), launch sequences of a
// crystal pass and of a cavity round trip, hipGraph replay, read-back.
#include "opo.h"
#include "kernel_list.h"
#include "schedule.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <unordered_set>
#include <vector>

namespace opo {

// the kernel instantiations live in the k_*.hip units
OPO_ALL_KERNELS(extern template)

static thread_local std::string g_err;

static int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

#define HIP_TRY(expr)                                                                            \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return fail(OPO_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));         \
    } while (0)

// Propagates a failed HIP call out of a function that returns hipError_t.
#define HIP_RET(expr)                                                                            \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess) return e_;                                                         \
    } while (0)

static constexpr int kHistChunk = 1024;   // round trips buffered on the device per read-back
static constexpr double kTwoPi = 6.283185307179586476925286766559;
static constexpr double kPi = 3.1415926535897932384626433832795;

struct Plan {
    int log2n1, log2n2, cols, rows;
};

static int ilog2(long long v)
{
    int l = 0;
    while ((1LL << l) < v) ++l;
    return l;
}

// Four-step split nt = n1 * n2: balanced up to 2^12, then columns of 64
// (short column transforms keep three fields of 128-byte column groups in
// registers) and rows up to the longest row kernel, then longer columns.
// col_log2 > 0 asks for columns of 2^col_log2 instead (for nt > 2^10, and
// never shorter than the longest rows allow, nor longer than balanced).
static Plan make_plan(int nt, int precision, int col_log2)
{
    Plan p;
    const int l = ilog2(nt);
    const int max_ln1 = precision == OPO_F64 ? kMaxLog2N1<double> : kMaxLog2N1<float>;
    if (col_log2 > 0 && l > 10) p.log2n2 = std::max(std::min(col_log2, l / 2), l - max_ln1);
    else if (l <= 12) p.log2n2 = l / 2;
    else p.log2n2 = std::max(6, l - max_ln1);
    p.log2n1 = l - p.log2n2;
    p.cols = precision == OPO_F64 ? col_cols<double>(p.log2n2) : col_cols<float>(p.log2n2);
    p.rows = precision == OPO_F64 ? row_rows<double>(p.log2n1) : row_rows<float>(p.log2n1);
    return p;
}

// A run of tiles that share one kernel instantiation.
struct Group {
    int ln;       // index of the size range
    int tile0;    // first tile
    int count;    // tiles
    int half;     // half of the batch (mixed schedule), 0 otherwise
    int nf;       // coupled waves of the group's instances (column groups)
    int only = 0; // 1 + the instance of every tile of the group, or 0
};

// StepArgs::inst_only of every group: whether all its tiles belong to one instance.
static void set_only(std::vector<Group> &groups, const std::vector<int> &tile_inst)
{
    for (Group &g : groups) {
        g.only = 0;
        if (g.count < 1) continue;
        const int first = tile_inst[g.tile0];
        bool one = true;
        for (int t = g.tile0; t < g.tile0 + g.count && one; ++t) one = tile_inst[t] == first;
        if (one) g.only = first + 1;
    }
}

// Index of the size range (kColRanges / kRowRanges) that contains ln.
template <size_t K> static int range_of(const int (&ranges)[K][2], int ln)
{
    for (size_t i = 0; i < K; ++i)
        if (ln >= ranges[i][0] && ln <= ranges[i][1]) return static_cast<int>(i);
    return -1;
}

template <typename R, int NF> static const void *column_fn_nf(int range)
{
    switch (range) {
    case 0: return reinterpret_cast<const void *>(&column_pass<R, kColRanges[0][0], kColRanges[0][1], NF>);
    case 1: return reinterpret_cast<const void *>(&column_pass<R, kColRanges[1][0], kColRanges[1][1], NF>);
    case 2: return reinterpret_cast<const void *>(&column_pass<R, kColRanges[2][0], kColRanges[2][1], NF>);
    default: return nullptr;
    }
}

template <typename R> static const void *column_fn(int range, int nf)
{
    return nf == 2 ? column_fn_nf<R, 2>(range) : column_fn_nf<R, 3>(range);
}

template <typename R> static const void *row_fn(int range)
{
    switch (range) {
    case 0: return reinterpret_cast<const void *>(&row_pass<R, kRowRanges[0][0], kRowRanges[0][1]>);
    case 1: return reinterpret_cast<const void *>(&row_pass<R, kRowRanges[1][0], kRowRanges[1][1]>);
    case 2:
        if constexpr (kMaxLog2N1<R> >= kRowRanges[2][0])
            return reinterpret_cast<const void *>(&row_pass<R, kRowRanges[2][0], kRowRanges[2][1]>);
        return nullptr;
    default: return nullptr;
    }
}

// Mixed column/row kernels for the (column range, row range) pairs that the
// four-step split produces.
template <typename R, int NF> static const void *mixed_fn_nf(int cr, int rr)
{
    const int key = cr * 3 + rr;
    switch (key) {
    case 0: return reinterpret_cast<const void *>(&mixed_pass<R, 0, 0, NF>);
    case 1: return reinterpret_cast<const void *>(&mixed_pass<R, 0, 1, NF>);
    case 2:
        if constexpr (kMaxLog2N1<R> >= kRowRanges[2][0])
            return reinterpret_cast<const void *>(&mixed_pass<R, 0, 2, NF>);
        return nullptr;
    case 4: return reinterpret_cast<const void *>(&mixed_pass<R, 1, 1, NF>);
    case 5:
        if constexpr (kMaxLog2N1<R> >= kRowRanges[2][0])
            return reinterpret_cast<const void *>(&mixed_pass<R, 1, 2, NF>);
        return nullptr;
    case 7: return reinterpret_cast<const void *>(&mixed_pass<R, 2, 1, NF>);
    case 8:
        if constexpr (kMaxLog2N1<R> >= kRowRanges[2][0])
            return reinterpret_cast<const void *>(&mixed_pass<R, 2, 2, NF>);
        return nullptr;
    default: return nullptr;
    }
}

// Resident pass for instances of 2^ln points and nf waves (kResMinLog2..kResMaxLog2).
template <typename R, int NF> static const void *resident_fn_nf(int ln)
{
    switch (ln) {
    case 10: return reinterpret_cast<const void *>(&resident_pass<R, 10, NF>);
    case 11: return reinterpret_cast<const void *>(&resident_pass<R, 11, NF>);
    case 12:
        if constexpr (kResMaxLog2<R> >= 12) return reinterpret_cast<const void *>(&resident_pass<R, 12, NF>);
        return nullptr;
    default: return nullptr;
    }
}
template <typename R> static const void *resident_fn(int ln, int nf)
{
    return nf == 2 ? resident_fn_nf<R, 2>(ln) : resident_fn_nf<R, 3>(ln);
}
static int resident_threads(int ln, int precision)
{
    if (precision == OPO_F64) return ln <= 10 ? res_threads<double, 10>() : res_threads<double, 11>();
    return ln <= 10 ? res_threads<float, 10>() : ln == 11 ? res_threads<float, 11>() : res_threads<float, 12>();
}
static bool resident_shape(int ln, int precision)
{
    return ln >= kResMinLog2 && ln <= (precision == OPO_F64 ? kResMaxLog2<double> : kResMaxLog2<float>);
}

// Mixed kernel for column range cr of nf-wave instances and row range rr.
template <typename R> static const void *mixed_fn(int cr, int rr, int nf)
{
    return nf == 2 ? mixed_fn_nf<R, 2>(cr, rr) : mixed_fn_nf<R, 3>(cr, rr);
}

} // namespace opo

using namespace opo;

struct opo_s {
    int precision = OPO_F32;
    int device = 0;
    int n_inst = 0;
    int nz = 1;                      // steps of the first crystal
    int n_stage = 1;                 // crystals per round trip
    int order = 2;                   // splitting order: 2 symmetrized, 4 triple jump
    std::vector<int> stage_nz;       // steps per pass of each crystal
    hipStream_t stream = nullptr;
    bool own_stream = false;
    void *state = nullptr;
    bool own_state = false;
    size_t state_bytes = 0;
    size_t elem = 8;                 // bytes per complex sample
    void *pump = nullptr;            // input-pump samples (pulsed pumps only)
    std::vector<InstDesc> inst;
    InstDesc *d_inst = nullptr;
    int tiles_a = 0, tiles_b = 0;
    std::vector<Group> groups_a, groups_b;   // tiles of one size range (and half), two-pass instances
    // resident instances: their column and row tiles follow those of the two-pass
    // instances (the adaptive step and the spectrum read-out run them), and
    // their fixed-step passes run in resident_pass launches, one group per
    // (log2 nt, nf) over d_res_inst[tile0 .. tile0 + count)
    std::vector<Group> res_groups_a, res_groups_b, res_launch;
    int *d_res_inst = nullptr;
    // the resident launches' branches of a pass or round trip: one stream and join
    // event per launch group, so the shapes run concurrently
    std::vector<hipStream_t> sides;
    std::vector<hipEvent_t> ev_join;
    hipEvent_t ev_fork = nullptr;
    bool mixed = false;              // two halves a launch apart, mixed launches
    int *d_map[2] = {nullptr, nullptr};  // workgroup -> tile maps of the two mixed launches
    int map_len[2] = {0, 0};
    int *d_tile_a = nullptr, *d_tile_b = nullptr;
    void *d_tw = nullptr;
    void *d_w4tab = nullptr;         // four-step twiddle tables, one per distinct (nt, n1)
    void *d_disp = nullptr;          // linear-propagator tables, one per distinct crystal/grid
    std::vector<int> disp_owner;     // instance whose parameters define each table
    double disp_mode = -1.0;         // step the tables hold: > 0 explicit dz, 0 = L/nz, < 0 none
    double *d_partial = nullptr;
    double *d_hist = nullptr;
    int *d_counter = nullptr;        // [0] history slot in the chunk, [1] round trips completed,
                                     // [2] stop flag, [3] non-finite boundary value (ssfm_kernels.h)
    void *d_snap = nullptr;          // state at the start of the current round trip
    void *d_record = nullptr;        // [record_cap][state] fields leaving the crystal per round trip
    int record_cap = 0;
    size_t lds_a = 0, lds_b = 0;
    double z = 0.0;
    std::vector<double> hist;        // [rows][n_inst][3]
    int hist_rows = 0;
    bool any_gdd = false, any_eom = false;
    int use_graph = 1;
    hipGraphExec_t graph = nullptr;
    void *spec_buf = nullptr;        // spectrum read-out (opo_get_fields, domain 1)
    // adaptive step: coarse and fine copies of the state, per-instance
    // propagator tables (coarse and fine step), control state, error partials
    void *a_uc = nullptr, *a_uf = nullptr, *a_tab = nullptr;
    AdaptState *d_actl = nullptr;
    double *d_apart = nullptr;
    int a_chunks = 0;
    hipGraphExec_t a_graph = nullptr;   // one attempt, replayed (reads everything from the device)
    std::vector<double> t_window;    // T of every instance [ps]
    std::vector<double> out_scale;   // [instance][3] output power per unit area and energy, see opo_get_power_history
    // profile option: event pairs of the launches since the last collection
    bool profile = false;
    std::vector<hipEvent_t> events;
    std::vector<int> ev_class;
    size_t ev_used = 0;
    double k_ms[OPO_K_CLASSES] = {};
    long long k_count[OPO_K_CLASSES] = {};
};

namespace opo {

// Live handles, so that a NULL, foreign or destroyed handle is reported as
// OPO_ESTATE instead of being dereferenced.
static std::mutex g_live_mu;
static std::unordered_set<const opo_t *> g_live;

static bool is_live(const opo_t *h)
{
    std::lock_guard<std::mutex> lk(g_live_mu);
    return h && g_live.count(h) != 0;
}

static bool finite3(const double *v)
{
    return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]);
}

// Triple-jump coefficients of the fourth-order composition: a = 1/(2 - 2^(1/3)),
// b = 1 - 2a (a + b + a = 1, 2a^3 + b^3 = 0).
constexpr double kTjA = 1.35120719195965763405;
constexpr double kTjB = -1.70241438391931526810;

// Coupled waves of an instance: 3 (pump, signal, idler; n_fields 0 or 3) or 2
// (pump and degenerate signal).
static int nfields(const opo_fields_t &f) { return f.n_fields == 2 ? 2 : 3; }

// Coupling coefficients (Sec. 2.1, kappa_x = 2 pi d_eff/(n_x lambda_x)) in
// 1/mm per V/m (pm/V over um, then per mm). Two waves: the signal keeps
// kappa_s; the pump takes 2 pi d_eff/(n_p lambda_s), which conserves
// n_p|A_p|^2 + n_s|A_s|^2 (kappa_p/2 at lambda_s = 2 lambda_p).
static void coupling(const opo_fields_t &f, double deff, double kappa[3])
{
    for (int x = 0; x < 3; ++x) kappa[x] = kTwoPi * deff / (f.n[x] * f.lambda_um[x]) * 1e-9;
    if (nfields(f) == 2) {
        kappa[0] = kTwoPi * deff / (f.n[0] * f.lambda_um[1]) * 1e-9;
        kappa[2] = 0.0;
    }
}

// Crystal-dependent descriptor fields: length, couplings (Sec. 2.1), the
// Eq. 5 dispersion coefficients, loss, mismatch and the Kerr coefficients.
static void set_crystal(InstDesc &d, const opo_fields_t &f, const opo_crystal_t &c)
{
    const double T = f.t_window_ps;
    d.length_mm = c.length_mm;
    coupling(f, c.deff_pm_per_v, d.kappa);
    for (int x = 0; x < 3; ++x) {
        // Eq. 5 phase per mm in revolutions for bin ks (w = 2 pi ks/T):
        // (-db1 w + b2 w^2/2 - b3 w^3/6)/(2 pi)
        const double b2 = c.b2_fs2_per_mm[x] * 1e-6, b3 = c.b3_fs3_per_mm[x] * 1e-9;
        d.disp[x][0] = -c.db1_ps_per_mm[x] / T;
        d.disp[x][1] = kPi * b2 / (T * T);
        d.disp[x][2] = -kTwoPi * kTwoPi * b3 / (6.0 * T * T * T);
        d.alpha_half[x] = 0.5 * c.alpha_per_mm[x];
    }
    d.dk_rev = c.dk_per_mm / kTwoPi;
    // Kerr term: gamma_x = (2 pi/lambda_x) n2 (n_x eps0 c/2), per mm
    d.kerr = c.n2_m2_per_w != 0.0;
    for (int x = 0; x < 3; ++x)
        d.gamma[x] = kTwoPi / (f.lambda_um[x] * 1e-6) * c.n2_m2_per_w *
                     (0.5 * f.n[x] * 8.8541878128e-12 * 299792458.0) * 1e-3;
}

// Descriptor of one instance from its inputs and four-step split: everything
// but the offsets into the batch's buffers (state, input pump, tables, tiles).
static void fill_desc(InstDesc &d, const opo_fields_t &f, const opo_crystal_t &c, const opo_cavity_t &k,
                      const Plan &p)
{
    std::memset(&d, 0, sizeof(d));
    d.nt = f.nt;
    d.log2nt = ilog2(d.nt);
    d.n1 = 1 << p.log2n1;
    d.log2n1 = p.log2n1;
    d.n2 = 1 << p.log2n2;
    d.log2n2 = p.log2n2;
    d.cols = p.cols;
    d.rows = p.rows;
    d.nf = nfields(f);
    d.pump_off = -1;
    d.pump_windows = f.pump_windows > 1 ? f.pump_windows : 1;
    d.tiles_a = (d.n1 + d.cols - 1) / d.cols;
    d.tiles_b = d.nf * ((d.n2 + d.rows - 1) / d.rows);
    for (int x = 0; x < d.nf; ++x) {
        if (k.resonant[x]) d.res_mask |= 1 << x;
        if (k.gdd_on[x] && k.gdd_fs2 != 0.0) d.gdd_mask |= 1 << x;
        if (k.eom_on[x] && k.eom_beta != 0.0) d.eom_mask |= 1 << x;
    }
    const double T = f.t_window_ps;
    set_crystal(d, f, c);
    for (int x = 0; x < 3; ++x) {
        const double sr = std::sqrt(k.refl[x]);
        d.mirror[x][0] = sr * std::cos(k.delta_rad[x]);
        d.mirror[x][1] = sr * std::sin(k.delta_rad[x]);
    }
    d.gdd_rev = kPi * k.gdd_fs2 * 1e-6 / (T * T);   // gamma w^2/2 / (2 pi)
    d.eom_beta = k.eom_beta;
    d.eom_rev0 = -0.5 * T * k.eom_fpm_thz;          // f t_0
    d.eom_rev_step = k.eom_fpm_thz * T / d.nt;       // f dt
    d.pump_cw[0] = f.pump_cw[0];
    d.pump_cw[1] = f.pump_cw[1];
    // a resonant pump: the input couples in through the pump mirror
    d.inject = k.resonant[0] ? std::sqrt(1.0 - k.refl[0]) : 0.0;
}

static int validate(int n, int K, const opo_fields_t *f, const opo_crystal_t *c, const opo_cavity_t *k,
                    int precision, double step_scale)
{
    const int max_log2 = precision == OPO_F64 ? 19 : 20;
    for (int i = 0; i < n; ++i) {
        const std::string at = "instance " + std::to_string(i) + ": ";
        const int nt = f[i].nt;
        if (nt < 2 || (nt & (nt - 1)) || ilog2(nt) > max_log2)
            return fail(OPO_EINVAL, at + "nt must be a power of two in [2, 2^" +
                                        std::to_string(max_log2) + "]");
        if (!(f[i].t_window_ps > 0.0) || !std::isfinite(f[i].t_window_ps))
            return fail(OPO_EINVAL, at + "t_window_ps must be finite and > 0");
        if (f[i].n_fields != 0 && f[i].n_fields != 2 && f[i].n_fields != 3)
            return fail(OPO_EINVAL, at + "n_fields must be 2, 3 or 0 (= 3)");
        const int nf = nfields(f[i]);
        for (int x = 0; x < nf; ++x)
            if (!(f[i].lambda_um[x] > 0.0) || !std::isfinite(f[i].lambda_um[x]) ||
                !(f[i].n[x] > 0.0) || !std::isfinite(f[i].n[x]))
                return fail(OPO_EINVAL, at + "wavelengths and indices must be finite and > 0");
        if (!std::isfinite(f[i].pump_cw[0]) || !std::isfinite(f[i].pump_cw[1]))
            return fail(OPO_EINVAL, at + "pump_cw must be finite");
        if (f[i].pump_windows < 0 || (f[i].pump_windows > 1 && !f[i].pump_in))
            return fail(OPO_EINVAL, at + "pump_windows must be >= 0, and > 1 only with pump_in");
        for (int st = 0; st < K; ++st) {
            const opo_crystal_t &cr = c[i * K + st];
            const std::string cat = K > 1 ? at + "crystal " + std::to_string(st) + ": " : at;
            if (!(cr.length_mm > 0.0) || !std::isfinite(cr.length_mm))
                return fail(OPO_EINVAL, cat + "length_mm must be finite and > 0");
            if (cr.nz < 1) return fail(OPO_EINVAL, cat + "nz must be >= 1");
            if (cr.nz != c[st].nz) return fail(OPO_EINVAL, cat + "all instances must share nz");
            if (!std::isfinite(cr.deff_pm_per_v) || !std::isfinite(cr.dk_per_mm) || !std::isfinite(cr.n2_m2_per_w) ||
                !finite3(cr.alpha_per_mm) || !finite3(cr.db1_ps_per_mm) || !finite3(cr.b2_fs2_per_mm) ||
                !finite3(cr.b3_fs3_per_mm))
                return fail(OPO_EINVAL, cat + "crystal coefficients must be finite");
        }
        for (int x = 0; x < 3; ++x) {
            if (!(k[i].refl[x] >= 0.0 && k[i].refl[x] <= 1.0))
                return fail(OPO_EINVAL, at + "reflectivities must lie in [0, 1]");
        }
        if (!finite3(k[i].delta_rad) || !std::isfinite(k[i].gdd_fs2) ||
            !std::isfinite(k[i].eom_beta) || !std::isfinite(k[i].eom_fpm_thz))
            return fail(OPO_EINVAL, at + "cavity parameters must be finite");

        // step criterion of Sec. 2.4: the nonlinear change per step,
        // kappa |A| dz, must stay well below one
        double amax = std::hypot(f[i].pump_cw[0], f[i].pump_cw[1]);
        if (f[i].init)
            for (long long q = 0; q < static_cast<long long>(nf) * nt; ++q)
                amax = std::max(amax, std::hypot(f[i].init[2 * q], f[i].init[2 * q + 1]));
        if (f[i].pump_in)
            for (long long q = 0; q < static_cast<long long>(nt) * std::max(1, f[i].pump_windows); ++q)
                amax = std::max(amax, std::hypot(f[i].pump_in[2 * q], f[i].pump_in[2 * q + 1]));
        if (!std::isfinite(amax)) return fail(OPO_EINVAL, at + "initial fields must be finite");
        for (int st = 0; st < K; ++st) {
            const opo_crystal_t &cr = c[i * K + st];
            double kap[3], kmax = 0.0;
            coupling(f[i], cr.deff_pm_per_v, kap);
            for (int x = 0; x < nf; ++x)
                kmax = std::max(kmax, std::fabs(kap[x]));
            const double step = kmax * amax * step_scale * cr.length_mm / cr.nz;
            if (!(step < 0.5))
                return fail(OPO_EINVAL, at + "step too large for the field amplitudes (kappa |A| dz = " +
                                            std::to_string(step) + ", needs < 0.5)");
        }
    }
    return OPO_OK;
}

// Unit-modulus factors computed in FP64, stored as Phasor<R> (compensated
// FP32 pairs, or FP64).
template <typename R> static hipError_t upload_phasors(void *dst, const std::vector<double> &re,
                                                       const std::vector<double> &im, hipStream_t st)
{
    std::vector<Phasor<R>> buf(re.size());
    for (size_t i = 0; i < re.size(); ++i)
        buf[i] = make_phasor<R>(re[i], im[i]);
    hipError_t e = hipMemcpyAsync(dst, buf.data(), buf.size() * sizeof(Phasor<R>), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(st);   // buf is released on return
}

template <typename R> static hipError_t host_to_state(void *dst, const double *src, long long count,
                                                      hipStream_t st)
{
    std::vector<R> buf(2 * count);
    for (long long i = 0; i < 2 * count; ++i)
        buf[i] = static_cast<R>(src[i]);
    hipError_t e = hipMemcpyAsync(dst, buf.data(), buf.size() * sizeof(R), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(st);
}

template <typename R> static hipError_t state_to_host(double *dst, const void *src, long long count,
                                                      hipStream_t st)
{
    std::vector<R> buf(2 * count);
    hipError_t e = hipMemcpyAsync(buf.data(), src, buf.size() * sizeof(R), hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    for (long long i = 0; i < 2 * count; ++i)
        dst[i] = static_cast<double>(buf[i]);
    return hipSuccess;
}

static void release(opo_t *h)
{
    if (!h) return;
    (void)hipSetDevice(h->device);
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    if (h->graph) (void)hipGraphExecDestroy(h->graph);
    if (h->a_graph) (void)hipGraphExecDestroy(h->a_graph);
    if (h->own_state && h->state) (void)hipFree(h->state);
    if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
    for (hipEvent_t e : h->ev_join)
        if (e) (void)hipEventDestroy(e);
    for (hipStream_t st : h->sides)
        if (st) (void)hipStreamDestroy(st);
    void *bufs[] = {h->d_res_inst, h->d_w4tab, h->pump, h->d_inst, h->d_tile_a, h->d_tile_b, h->d_tw, h->d_disp, h->d_map[0], h->d_map[1],
                    h->d_partial, h->d_hist, h->d_counter, h->spec_buf, h->d_record, h->d_snap,
                    h->a_uc, h->a_uf, h->a_tab, h->d_actl, h->d_apart};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    for (hipEvent_t e : h->events)
        if (e) (void)hipEventDestroy(e);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
    {
        std::lock_guard<std::mutex> lk(g_live_mu);
        g_live.erase(h);
    }
    delete h;
}

template <typename R> static StepArgs<R> base_args(opo_t *h, void *state)
{
    StepArgs<R> a{};
    a.inst = h->d_inst;
    a.state = static_cast<cplx<R> *>(state);
    a.pump = static_cast<const cplx<R> *>(h->pump);
    a.tw = static_cast<const Phasor<R> *>(h->d_tw);
    a.w4tab = static_cast<const Phasor<R> *>(h->d_w4tab);
    a.disp = static_cast<const Phasor<R> *>(h->d_disp);
    a.partial = h->d_partial;
    a.counter = h->d_counter;
    a.record = static_cast<cplx<R> *>(h->d_record);
    a.record_stride = static_cast<long long>(h->state_bytes / h->elem);
    a.record_cap = h->record_cap;
    a.nz = h->nz;
    return a;
}

static void substep(const opo_t *h, int i, double &z, double &tau, int &sel)
{
    if (h->order != 4) {
        z = i;
        tau = 1.0;
        sel = 0;
        return;
    }
    const int j = i >= 0 ? i / 3 : -1, s = i - 3 * j;
    const double start[3] = {0.0, kTjA, kTjA + kTjB}, size[3] = {kTjA, kTjB, kTjA};
    z = j + start[s];
    tau = size[s];
    sel = s == 1 ? 1 : 0;
}

// profile option: open an event pair around the next launch of class k
static hipError_t prof_begin(opo_t *h, int k)
{
    if (!h->profile) return hipSuccess;
    if (h->ev_used + 2 > h->events.size()) {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        HIP_RET(hipEventCreate(&e0));
        hipError_t e = hipEventCreate(&e1);
        if (e != hipSuccess) {
            (void)hipEventDestroy(e0);   // already failing: the first error is the one reported
            return e;
        }
        h->events.push_back(e0);
        h->events.push_back(e1);
        h->ev_class.push_back(k);
    }
    h->ev_class[h->ev_used / 2] = k;
    return hipEventRecord(h->events[h->ev_used], h->stream);
}

static hipError_t prof_end(opo_t *h)
{
    if (!h->profile) return hipSuccess;
    HIP_RET(hipEventRecord(h->events[h->ev_used + 1], h->stream));
    h->ev_used += 2;
    return hipSuccess;
}

// profile option: wait for the recorded launches and add up the times of the
// first `used` events
static int prof_collect(opo_t *h, size_t used)
{
    if (!h->profile || used == 0) return OPO_OK;
    HIP_TRY(hipStreamSynchronize(h->stream));
    for (size_t i = 0; i < used; i += 2) {
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, h->events[i], h->events[i + 1]));
        h->k_ms[h->ev_class[i / 2]] += ms;
        h->k_count[h->ev_class[i / 2]] += 1;
    }
    return OPO_OK;
}

// Step i of a pass in units of dz: start z, size tau, and the propagator
// table it uses. Symmetrized steps are the steps; the fourth-order
// composition runs three per step, of a, b and a times dz.
static void substep(const opo_t *h, int i, double &z, double &tau, int &sel);

// The RK4 half-steps a column launch at step boundary i runs: the second
// half of step i-1 and the first half of step i.
template <typename R> static void set_half_steps(const opo_t *h, StepArgs<R> &a, int i)
{
    double z, tau;
    int sel;
    substep(h, i - 1, z, tau, sel);
    a.zf_prev = z + 0.5 * tau;
    a.hf_prev = 0.5 * tau;
    substep(h, i, z, tau, sel);
    a.zf_this = z;
    a.hf_this = 0.5 * tau;
}

// Column launches over the two-pass instances (of one half, or all), and with
// all_tiles also over the tiles of the resident instances (the adaptive step
// and the spectrum read-out).
template <typename R>
static hipError_t launch_a(opo_t *h, StepArgs<R> a, int flags, int step, int half = -1, bool all_tiles = false)
{
    a.tile_inst = h->d_tile_a;
    a.flags = flags;
    set_half_steps<R>(h, a, step);
    HIP_RET(prof_begin(h, OPO_K_COLUMN));
    for (int set = 0; set < (all_tiles ? 2 : 1); ++set)
        for (const Group &g : set ? h->res_groups_a : h->groups_a) {
            if (half >= 0 && g.half != half) continue;
            a.tile0 = g.tile0;
            a.tile_count = g.count;
            a.inst_only = g.only;
            void *args[] = {&a};
            HIP_RET(hipLaunchKernel(column_fn<R>(g.ln, g.nf), dim3(g.count), dim3(kThreads), args, h->lds_a,
                                    h->stream));
        }
    return prof_end(h);
}

template <typename R>
static hipError_t launch_b(opo_t *h, StepArgs<R> a, int flags, int step = 0, int sel = -1, bool all_tiles = false)
{
    a.tile_inst = h->d_tile_b;
    a.flags = flags;
    double z, tau;
    substep(h, step, z, tau, a.disp_sel);
    if (sel >= 0) a.disp_sel = sel;
    HIP_RET(prof_begin(h, OPO_K_ROW));
    for (int set = 0; set < (all_tiles ? 2 : 1); ++set)
        for (const Group &g : set ? h->res_groups_b : h->groups_b) {
            a.tile0 = g.tile0;
            a.tile_count = g.count;
            a.inst_only = g.only;
            void *args[] = {&a};
            HIP_RET(hipLaunchKernel(row_fn<R>(g.ln), dim3(g.count), dim3(kThreads), args, h->lds_b, h->stream));
        }
    return prof_end(h);
}

// The resident launches of a pass (flags as in resident_pass): one per shape,
// each on its own side stream between the fork event and its join event
// (parallel branches of the captured graph, which the shapes fill side by side),
// or all on the handle's stream under the profile option.
template <typename R> static hipError_t launch_resident(opo_t *h, StepArgs<R> a, int flags)
{
    if (h->res_launch.empty()) return hipSuccess;
    if (!h->profile) HIP_RET(hipEventRecord(h->ev_fork, h->stream));
    a.tile_inst = h->d_res_inst;
    a.flags = flags;
    HIP_RET(prof_begin(h, OPO_K_RESIDENT));
    for (size_t q = 0; q < h->res_launch.size(); ++q) {
        const Group &g = h->res_launch[q];
        hipStream_t st = h->profile ? h->stream : h->sides[q];
        if (!h->profile) HIP_RET(hipStreamWaitEvent(st, h->ev_fork, 0));
        a.tile0 = g.tile0;
        a.tile_count = g.count;
        const int prec = sizeof(R) == 8 ? OPO_F64 : OPO_F32;
        const size_t lds = static_cast<size_t>(lds_elems<R>(1 << g.ln)) * sizeof(cplx<R>);
        void *args[] = {&a};
        HIP_RET(hipLaunchKernel(resident_fn<R>(g.ln, g.nf), dim3(g.count), dim3(resident_threads(g.ln, prec)), args,
                                lds, st));
        if (!h->profile) HIP_RET(hipEventRecord(h->ev_join[q], st));
    }
    return prof_end(h);
}

// The handle's stream waits for the resident branches (before the energies).
static hipError_t join_resident(opo_t *h)
{
    if (h->res_launch.empty() || h->profile) return hipSuccess;
    for (hipEvent_t e : h->ev_join)
        HIP_RET(hipStreamWaitEvent(h->stream, e, 0));
    return hipSuccess;
}

// Column tiles of half `ch` (flags, step) with the row tiles (B_DISP) of the
// other half, in one launch.
template <typename R> static hipError_t launch_mixed(opo_t *h, StepArgs<R> a, int ch, int cflags, int step)
{
    const Group &gc = h->groups_a[ch], &gr = h->groups_b[1 - ch];
    StepArgs<R> ac = a, ar = a;
    ac.tile_inst = h->d_tile_a;
    ac.flags = cflags;
    set_half_steps<R>(h, ac, step);
    ac.tile0 = gc.tile0;
    ac.tile_count = gc.count;
    ac.block_map = h->d_map[ch];
    ar.tile_inst = h->d_tile_b;
    ar.flags = B_DISP;
    {
        // the other half is a launch ahead (half 0) or behind (half 1)
        double z, tau;
        substep(h, ch == 1 ? step : step - 1, z, tau, ar.disp_sel);
    }
    ar.tile0 = gr.tile0;
    ar.tile_count = gr.count;
    void *args[] = {&ac, &ar};
    HIP_RET(prof_begin(h, OPO_K_MIXED));
    HIP_RET(hipLaunchKernel(mixed_fn<R>(gc.ln, gr.ln, gc.nf), dim3(h->map_len[ch]), dim3(kThreads), args,
                            std::max(h->lds_a, h->lds_b), h->stream));
    return prof_end(h);
}

// One crystal pass of nz steps. `first` flags are OR-ed into the opening
// column pass (refresh), `last` into the closing one (energy, mirror, EOM).
template <typename R>
static hipError_t enqueue_pass(opo_t *h, StepArgs<R> a, int nz_steps, int first, int last)
{
    if (h->groups_a.empty()) return hipSuccess;           // every instance is resident
    const int nz = nz_steps * (h->order == 4 ? 3 : 1);   // symmetrized steps of the pass
    if (h->mixed) {
        // half 0 runs one launch ahead of half 1
        const int mid = A_INV | A_RK_PREV | A_RK_THIS | A_FWD;
        HIP_RET(launch_a<R>(h, a, first | A_RK_THIS | A_FWD, 0, 0));
        for (int j = 0; j < nz; ++j) {
            HIP_RET(launch_mixed<R>(h, a, 1, j == 0 ? (first | A_RK_THIS | A_FWD) : mid, j));      // rows of half 0
            HIP_RET(launch_mixed<R>(h, a, 0, j + 1 < nz ? mid : (A_INV | A_RK_PREV | last), j + 1));  // rows of half 1
        }
        return launch_a<R>(h, a, A_INV | A_RK_PREV | last, nz, 1);
    }
    HIP_RET(launch_a<R>(h, a, first | A_RK_THIS | A_FWD, 0));
    for (int j = 0; j < nz; ++j) {
        HIP_RET(launch_b<R>(h, a, B_DISP, j));
        if (j + 1 < nz) HIP_RET(launch_a<R>(h, a, A_INV | A_RK_PREV | A_RK_THIS | A_FWD, j + 1));
        else HIP_RET(launch_a<R>(h, a, A_INV | A_RK_PREV | last, nz));
    }
    return hipSuccess;
}

// One cavity round trip (loop order of Sec. 4.1). Its refresh launch keeps
// the state it starts from in d_snap.
template <typename R> static hipError_t enqueue_roundtrip(opo_t *h)
{
    StepArgs<R> a = base_args<R>(h, h->state);
    a.dz_arg = 0.0;
    a.zbase = 0.0;
    a.snap = static_cast<cplx<R> *>(h->d_snap);
    const int eom = h->any_eom ? A_EOM : 0;
    const int K = h->n_stage;
    // resident instances (one crystal only): the whole round trip in one launch
    // per shape, beside the two-pass launches
    a.inst = h->d_inst;
    a.nz = h->stage_nz[0];
    HIP_RET(launch_resident<R>(h, a, A_REFRESH | A_ENERGY | (h->any_gdd ? A_GDD : 0) | A_MIRROR | eom));
    // the crystals in order, each from its own entrance; the boundary after the last
    for (int st = 0; st < K; ++st) {
        a.inst = h->d_inst + static_cast<size_t>(st) * h->n_inst;
        a.nz = h->stage_nz[st];
        const int first = st == 0 ? A_REFRESH : 0;
        if (st + 1 < K) {
            HIP_RET(enqueue_pass<R>(h, a, a.nz, first, 0));
        } else if (h->any_gdd && !h->groups_a.empty()) {
            HIP_RET(enqueue_pass<R>(h, a, a.nz, first, A_ENERGY | A_FWD));
            HIP_RET(launch_b<R>(h, a, B_GDD));
            HIP_RET(launch_a<R>(h, a, A_INV | A_MIRROR | eom, 0));
        } else {
            HIP_RET(enqueue_pass<R>(h, a, a.nz, first, A_ENERGY | A_MIRROR | eom));
        }
    }
    HIP_RET(join_resident(h));
    HIP_RET(prof_begin(h, OPO_K_ENERGY));
    energy_reduce<<<1, kThreads, 0, h->stream>>>(h->d_inst, h->n_inst, h->d_partial, h->d_hist,
                                                 h->d_counter, kHistChunk);
    HIP_RET(hipGetLastError());
    return prof_end(h);
}

template <typename R> static int setup_kernels(opo_t *h)
{
    for (const Group &g : h->groups_a) {
        if (!column_fn<R>(g.ln, g.nf)) return fail(OPO_EINVAL, "internal: no column kernel for this size");
        HIP_TRY(hipFuncSetAttribute(column_fn<R>(g.ln, g.nf), hipFuncAttributeMaxDynamicSharedMemorySize,
                                    static_cast<int>(h->lds_a)));
    }
    for (const Group &g : h->groups_b) {
        if (!row_fn<R>(g.ln)) return fail(OPO_EINVAL, "internal: no row kernel for this size");
        HIP_TRY(hipFuncSetAttribute(row_fn<R>(g.ln), hipFuncAttributeMaxDynamicSharedMemorySize,
                                    static_cast<int>(h->lds_b)));
    }
    for (const Group &g : h->res_groups_a)
        HIP_TRY(hipFuncSetAttribute(column_fn<R>(g.ln, g.nf), hipFuncAttributeMaxDynamicSharedMemorySize,
                                    static_cast<int>(h->lds_a)));
    for (const Group &g : h->res_groups_b)
        HIP_TRY(hipFuncSetAttribute(row_fn<R>(g.ln), hipFuncAttributeMaxDynamicSharedMemorySize,
                                    static_cast<int>(h->lds_b)));
    for (const Group &g : h->res_launch) {
        if (!resident_fn<R>(g.ln, g.nf)) return fail(OPO_EINVAL, "internal: no resident kernel for this size");
        HIP_TRY(hipFuncSetAttribute(resident_fn<R>(g.ln, g.nf), hipFuncAttributeMaxDynamicSharedMemorySize,
                                    static_cast<int>(lds_elems<R>(1 << g.ln) * sizeof(cplx<R>))));
    }
    if (h->mixed)
        for (int hf = 0; hf < 2; ++hf) {
            const Group &gc = h->groups_a[1 - hf];
            HIP_TRY(hipFuncSetAttribute(mixed_fn<R>(gc.ln, h->groups_b[hf].ln, gc.nf),
                                        hipFuncAttributeMaxDynamicSharedMemorySize,
                                        static_cast<int>(std::max(h->lds_a, h->lds_b))));
        }
    return OPO_OK;
}

static int init_impl(opo_t **out, int n, const opo_fields_t *f, const opo_crystal_t *c,
                     const opo_cavity_t *k, const opo_options_t *opt_in)
{
    opo_options_t opt{};
    if (opt_in) opt = *opt_in;
    // HIP cannot time events recorded inside a captured graph: the profile
    // option runs the round trip as plain launches
    if (opt.profile) opt.use_graph = -1;
    if (opt.precision != OPO_F32 && opt.precision != OPO_F64)
        return fail(OPO_EINVAL, "precision must be OPO_F32 or OPO_F64");
    if (opt.record_rt < 0) return fail(OPO_EINVAL, "record_rt must be >= 0");
    const int K = opt.n_crystals > 1 ? opt.n_crystals : 1;
    if (opt.n_crystals < 0) return fail(OPO_EINVAL, "n_crystals must be >= 0");
    if (opt.col_log2 != 0 && (opt.col_log2 < 4 || opt.col_log2 > kMaxLog2N2))
        return fail(OPO_EINVAL, "col_log2 must be 0 or 4.." + std::to_string(kMaxLog2N2));
    if (opt.schedule < 0 || opt.schedule > 2) return fail(OPO_EINVAL, "schedule must be 0, 1 or 2");
    if (opt.split_order != 0 && opt.split_order != 2 && opt.split_order != 4)
        return fail(OPO_EINVAL, "split_order must be 2, 4 or 0 (= 2)");
    // the longest symmetrized step of the fourth-order composition is |b| dz
    int rc = validate(n, K, f, c, k, opt.precision, opt.split_order == 4 ? -kTjB : 1.0);
    if (rc) return rc;

    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= opt.device || opt.device < 0)
        return fail(OPO_EDEVICE, "no HIP device with ordinal " + std::to_string(opt.device));
    HIP_TRY(hipSetDevice(opt.device));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, opt.device));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(OPO_EDEVICE, std::string("device is ") + prop.gcnArchName + ", library built for gfx950");

    opo_t *h = new (std::nothrow) opo_s();
    if (!h) return fail(OPO_ENOMEM, "handle allocation failed");
    h->precision = opt.precision;
    h->device = opt.device;
    h->n_inst = n;
    h->nz = c[0].nz;
    h->n_stage = K;
    h->order = opt.split_order == 4 ? 4 : 2;
    for (int st = 0; st < K; ++st) h->stage_nz.push_back(c[st].nz);
    h->elem = opt.precision == OPO_F64 ? 16 : 8;
    h->use_graph = opt.use_graph >= 0 ? 1 : 0;
    h->profile = opt.profile != 0;

    auto bail = [&](int code) {
        release(h);
        return code;
    };

    if (opt.stream) {
        h->stream = static_cast<hipStream_t>(opt.stream);
    } else {
        if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess)
            return bail(fail(OPO_EDEVICE, "hipStreamCreate failed"));
        h->own_stream = true;
    }

    // ---- plan and per-instance descriptors
    const uint64_t need = opo_state_bytes(n, f, opt.precision);
    long long off = 0, pump_elems = 0;
    std::map<std::pair<int, int>, long long> w4map;   // (log2 nt, log2 n1) -> four-step table offset
    long long w4_elems = 0;
    std::vector<int> tile_a_inst, tile_b_inst;
    size_t max_a = 0, max_b = 0;
    h->inst.resize(n);
    // the table's batch entries apply when the handle's fields fill the chip
    long long total_points = 0;
    for (int i = 0; i < n; ++i) total_points += static_cast<long long>(nfields(f[i])) * f[i].nt;
    const bool batched = total_points >= kBatchPoints;
    for (int i = 0; i < n; ++i) {
        InstDesc &d = h->inst[i];
        // schedule: the table's entry for this shape (schedule 0), or two-pass
        // (1) / resident where served (2); an explicit col_log2 sets the split
        const int l2 = ilog2(f[i].nt);
        const Schedule sc = opt.schedule == 0 ? schedule_lookup(opt.precision == OPO_F64, nfields(f[i]), l2, batched)
                                              : Schedule{0, opt.schedule == 2 ? 1 : 0};
        const Plan p = make_plan(f[i].nt, opt.precision, opt.col_log2 != 0 ? opt.col_log2 : sc.col_log2);
        fill_desc(d, f[i], c[i * K], k[i], p);
        // resident passes: shapes resident_pass serves, second-order steps, one crystal
        d.resident = sc.resident && resident_shape(l2, opt.precision) && h->order == 2 && K == 1 ? 1 : 0;
        d.off = off;
        off += static_cast<long long>(d.nf) * d.nt;
        if (f[i].pump_in) {
            d.pump_off = pump_elems;
            pump_elems += static_cast<long long>(d.nt) * d.pump_windows;
        }
        // LDS of a tile: nf fields of `cols` columns in rows of cols + 1 elements
        // (col_lds_row), or `rows` rows
        const bool seq = opt.precision == OPO_F64 ? col_seq_lds<double>(p.log2n2) : col_seq_lds<float>(p.log2n2);
        const int row = opt.precision == OPO_F64 ? col_lds_row<double>(p.log2n2) : col_lds_row<float>(p.log2n2);
        max_a = std::max(max_a, static_cast<size_t>(seq ? 1 : d.nf) * row * d.n2);
        max_b = std::max(max_b, static_cast<size_t>(d.rows) * d.n1);
        // shapes the kernels are instantiated for
        const int max_ln1 = opt.precision == OPO_F64 ? kMaxLog2N1<double> : kMaxLog2N1<float>;
        if (p.log2n2 > kMaxLog2N2 || p.log2n1 > max_ln1 || d.n1 > kTwL || d.n2 > kTwL ||
            static_cast<long long>(d.n1) * d.n2 != d.nt || d.cols < 1 || d.rows < 1)
            return bail(fail(OPO_EINVAL, "internal: tile plan out of bounds for nt " + std::to_string(d.nt)));

        // four-step twiddles W_nt^{j1 k2}: one table per distinct (nt, n1)
        {
            const std::pair<int, int> key(d.log2nt, d.log2n1);
            auto it = w4map.find(key);
            if (it == w4map.end()) {
                it = w4map.emplace(key, w4_elems).first;
                w4_elems += d.nt;
            }
            d.w4_off = it->second;
        }

        h->any_gdd |= d.gdd_mask != 0;
        h->any_eom |= d.eom_mask != 0;
    }

    // ---- halves of a batch for the mixed schedule: instances are dealt to
    // two halves of similar size (largest first); the schedule is used when
    // each half then has one column and one row size range (a GDD row pass
    // and the column pass after it run over both halves at the round-trip end)
    std::vector<int> half(n, 0);
    std::vector<int> order;
    for (int i = 0; i < n; ++i)
        if (!h->inst[i].resident) order.push_back(i);
    if (order.size() >= 2) {
        std::stable_sort(order.begin(), order.end(),
                         [&](int x, int y) { return h->inst[x].nt > h->inst[y].nt; });
        long long load[2] = {0, 0};
        for (int i : order) {
            const int hf = load[0] <= load[1] ? 0 : 1;
            half[i] = hf;
            load[hf] += h->inst[i].nt;
        }
    }
    // ---- tiles grouped by half and size range, one launch per group
    constexpr int ncr = sizeof(kColRanges) / sizeof(kColRanges[0]);
    constexpr int nrr = sizeof(kRowRanges) / sizeof(kRowRanges[0]);
    for (int hf = 0; hf < 2; ++hf)
        for (int nf = 3; nf >= 2; --nf)
            for (int g = 0; g < ncr; ++g) {
                const int first = h->tiles_a;
                for (int i = 0; i < n; ++i) {
                    InstDesc &d = h->inst[i];
                    if (d.resident || half[i] != hf || d.nf != nf || range_of(kColRanges, d.log2n2) != g) continue;
                    d.tile_a0 = h->tiles_a;
                    h->tiles_a += d.tiles_a;
                    tile_a_inst.insert(tile_a_inst.end(), d.tiles_a, i);
                }
                if (h->tiles_a > first) h->groups_a.push_back({g, first, h->tiles_a - first, hf, nf});
            }
    for (int hf = 0; hf < 2; ++hf)
        for (int g = 0; g < nrr; ++g) {
            const int first = h->tiles_b;
            for (int i = 0; i < n; ++i) {
                InstDesc &d = h->inst[i];
                if (d.resident || half[i] != hf || range_of(kRowRanges, d.log2n1) != g) continue;
                d.tile_b0 = h->tiles_b;
                h->tiles_b += d.tiles_b;
                tile_b_inst.insert(tile_b_inst.end(), d.tiles_b, i);
            }
            if (h->tiles_b > first) h->groups_b.push_back({g, first, h->tiles_b - first, hf, 0});
        }
    // the resident instances' tiles follow, and their launch groups by (log2 nt, nf)
    std::vector<int> res_inst;
    for (int nf = 3; nf >= 2; --nf)
        for (int g = 0; g < ncr; ++g) {
            const int first = h->tiles_a;
            for (int i = 0; i < n; ++i) {
                InstDesc &d = h->inst[i];
                if (!d.resident || d.nf != nf || range_of(kColRanges, d.log2n2) != g) continue;
                d.tile_a0 = h->tiles_a;
                h->tiles_a += d.tiles_a;
                tile_a_inst.insert(tile_a_inst.end(), d.tiles_a, i);
            }
            if (h->tiles_a > first) h->res_groups_a.push_back({g, first, h->tiles_a - first, 0, nf});
        }
    for (int g = 0; g < nrr; ++g) {
        const int first = h->tiles_b;
        for (int i = 0; i < n; ++i) {
            InstDesc &d = h->inst[i];
            if (!d.resident || range_of(kRowRanges, d.log2n1) != g) continue;
            d.tile_b0 = h->tiles_b;
            h->tiles_b += d.tiles_b;
            tile_b_inst.insert(tile_b_inst.end(), d.tiles_b, i);
        }
        if (h->tiles_b > first) h->res_groups_b.push_back({g, first, h->tiles_b - first, 0, 0});
    }
    for (int ln = kResMaxLog2<float>; ln >= kResMinLog2; --ln)
        for (int nf = 3; nf >= 2; --nf) {
            const int first = static_cast<int>(res_inst.size());
            for (int i = 0; i < n; ++i)
                if (h->inst[i].resident && h->inst[i].nf == nf && h->inst[i].log2nt == ln) res_inst.push_back(i);
            const int cnt = static_cast<int>(res_inst.size()) - first;
            if (cnt > 0) h->res_launch.push_back({ln, first, cnt, 0, nf});
        }
    if (static_cast<int>(tile_a_inst.size()) != h->tiles_a || static_cast<int>(tile_b_inst.size()) != h->tiles_b)
        return bail(fail(OPO_EINVAL, "internal: a transform length has no kernel"));
    set_only(h->groups_a, tile_a_inst);
    set_only(h->groups_b, tile_b_inst);
    set_only(h->res_groups_a, tile_a_inst);
    set_only(h->res_groups_b, tile_b_inst);
    if (n >= 2 && h->groups_a.size() == 2 && h->groups_b.size() == 2 &&
        h->groups_a[0].half == 0 && h->groups_a[1].half == 1 && h->groups_b[0].half == 0 &&
        h->groups_b[1].half == 1) {
        const bool f64 = opt.precision == OPO_F64;
        h->mixed = true;
        for (int hf = 0; hf < 2; ++hf) {
            const Group &gc = h->groups_a[1 - hf];
            const void *fn = f64 ? mixed_fn<double>(gc.ln, h->groups_b[hf].ln, gc.nf)
                                 : mixed_fn<float>(gc.ln, h->groups_b[hf].ln, gc.nf);
            h->mixed = h->mixed && fn != nullptr;
        }
    }

    // ---- workgroup -> tile maps of the mixed launches. Workgroup b runs on
    // XCD b mod 8; row tile t of an instance goes to XCD t mod 8, column
    // tiles are spread evenly, and within an XCD the two kinds alternate in
    // proportion to their counts, the longer rows first
    // Measured orders (MI355X, ms per round trip): the kinds interleaved in
    // proportion to their counts with the longer rows first in each XCD (below)
    // ran the batched sweep 0.7 % faster than unsorted; all row tiles first ran
    // a batch of 2^16 instances 7 % and the two-wave sweep 6 % faster but the
    // batched sweep 1 % and batches of 2^13..2^15 2-3 % slower; column tiles
    // first was slower on the batched sweep too.
    std::vector<int> maps[2];
    if (h->mixed) {
        constexpr int kXcd = 8;
        for (int ch = 0; ch < 2; ++ch) {
            const Group &gc = h->groups_a[ch], &gr = h->groups_b[1 - ch];
            std::vector<int> qc[kXcd], qr[kXcd];
            for (int t = 0; t < gc.count; ++t) qc[t % kXcd].push_back(gc.tile0 + t);
            for (int t = 0; t < gr.count; ++t) {
                const int tile = gr.tile0 + t;
                const int local = tile - h->inst[tile_b_inst[tile]].tile_b0;
                qr[local % kXcd].push_back(tile);
            }
            // longer rows first within each XCD (stable: tile order otherwise)
            for (int x = 0; x < kXcd; ++x)
                std::stable_sort(qr[x].begin(), qr[x].end(), [&](int p, int q) {
                    return h->inst[tile_b_inst[p]].log2n1 > h->inst[tile_b_inst[q]].log2n1;
                });
            size_t len = 0;
            for (int x = 0; x < kXcd; ++x) len = std::max(len, qc[x].size() + qr[x].size());
            maps[ch].assign(len * kXcd, kNoTile);
            for (int x = 0; x < kXcd; ++x) {
                const long long nc = static_cast<long long>(qc[x].size());
                const long long tot = nc + static_cast<long long>(qr[x].size());
                for (long long q = 0; q < tot; ++q) {
                    const long long before = q * nc / tot;
                    const bool col = (q + 1) * nc / tot > before;
                    maps[ch][q * kXcd + x] = col ? qc[x][before] : -1 - qr[x][q - before];
                }
            }
            h->map_len[ch] = static_cast<int>(maps[ch].size());
        }
    }

    // ---- one descriptor per (crystal, instance): the crystals of a round trip
    // share everything but the crystal-dependent fields
    h->inst.resize(static_cast<size_t>(K) * n);
    for (int st = 1; st < K; ++st)
        for (int i = 0; i < n; ++i) {
            InstDesc &d = h->inst[static_cast<size_t>(st) * n + i];
            d = h->inst[i];
            set_crystal(d, f[i], c[i * K + st]);
        }

    // ---- linear-propagator tables: descriptors with the same grid, crystal
    // length, step count and dispersion share one table
    long long disp_elems = 0;
    for (int q = 0; q < K * n; ++q) {
        InstDesc &d = h->inst[q];
        int same = -1;
        for (int o : h->disp_owner) {
            const InstDesc &e = h->inst[o];
            if (e.nt == d.nt && e.nf == d.nf && e.resident == d.resident && e.length_mm == d.length_mm &&
                h->stage_nz[o / n] == h->stage_nz[q / n] &&
                std::memcmp(e.disp, d.disp, sizeof(d.disp)) == 0 &&
                std::memcmp(e.alpha_half, d.alpha_half, sizeof(d.alpha_half)) == 0) {
                same = o;
                break;
            }
        }
        if (same >= 0) {
            d.disp_off = h->inst[same].disp_off;
        } else {
            d.disp_off = disp_elems;
            disp_elems += static_cast<long long>(d.nf) * d.nt * (h->order == 4 ? 2 : 1);
            h->disp_owner.push_back(q);
        }
    }

    // ---- device memory
    if (opt.state) {
        if (opt.state_bytes < need)
            return bail(fail(OPO_EINVAL, "caller state buffer is smaller than opo_state_bytes()"));
        h->state = opt.state;
    } else {
        if (hipMalloc(&h->state, need) != hipSuccess)
            return bail(fail(OPO_ENOMEM, "hipMalloc of the field state failed"));
        h->own_state = true;
    }
    h->state_bytes = need;
    const size_t es = h->elem;
    if (pump_elems && hipMalloc(&h->pump, pump_elems * es) != hipSuccess)
        return bail(fail(OPO_ENOMEM, "hipMalloc of the input pump failed"));
    if (opt.record_rt > 0) {
        if (hipMalloc(&h->d_record, static_cast<size_t>(opt.record_rt) * need) != hipSuccess)
            return bail(fail(OPO_ENOMEM, "hipMalloc of the round-trip record failed"));
        h->record_cap = opt.record_rt;
        // slots of round trips that never ran here (before a restored position) read as zeros
        if (hipMemsetAsync(h->d_record, 0, static_cast<size_t>(opt.record_rt) * need, h->stream) != hipSuccess)
            return bail(fail(OPO_EDEVICE, "clearing the round-trip record failed"));
    }
    if (hipMalloc(&h->d_snap, need) != hipSuccess)
        return bail(fail(OPO_ENOMEM, "hipMalloc of the round-trip snapshot failed"));
    if (hipMalloc(reinterpret_cast<void **>(&h->d_inst), h->inst.size() * sizeof(InstDesc)) != hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&h->d_tile_a), h->tiles_a * sizeof(int)) != hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&h->d_tile_b), h->tiles_b * sizeof(int)) != hipSuccess ||
        hipMalloc(&h->d_tw, static_cast<size_t>(kTwEntries) * 16) != hipSuccess ||
        hipMalloc(&h->d_w4tab, static_cast<size_t>(w4_elems) * 16) != hipSuccess ||
        hipMalloc(&h->d_disp, static_cast<size_t>(disp_elems) * 16) != hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&h->d_partial), h->tiles_a * 3 * sizeof(double)) != hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&h->d_hist),
                  static_cast<size_t>(kHistChunk) * n * 3 * sizeof(double)) != hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&h->d_counter), 4 * sizeof(int)) != hipSuccess ||
        (h->mixed && (hipMalloc(reinterpret_cast<void **>(&h->d_map[0]), maps[0].size() * sizeof(int)) != hipSuccess ||
                      hipMalloc(reinterpret_cast<void **>(&h->d_map[1]), maps[1].size() * sizeof(int)) != hipSuccess)))
        return bail(fail(OPO_ENOMEM, "hipMalloc of the tables failed"));

    if (!res_inst.empty()) {
        if (hipMalloc(reinterpret_cast<void **>(&h->d_res_inst), res_inst.size() * sizeof(int)) != hipSuccess)
            return bail(fail(OPO_ENOMEM, "hipMalloc of the resident instance list failed"));
        if (hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming) != hipSuccess)
            return bail(fail(OPO_EDEVICE, "creating the resident branches' fork event failed"));
        h->sides.assign(h->res_launch.size(), nullptr);
        h->ev_join.assign(h->res_launch.size(), nullptr);
        for (size_t q = 0; q < h->res_launch.size(); ++q)
            if (hipStreamCreateWithFlags(&h->sides[q], hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&h->ev_join[q], hipEventDisableTiming) != hipSuccess)
                return bail(fail(OPO_EDEVICE, "creating the resident branches' streams and events failed"));
    }

    h->lds_a = max_a * es;
    h->lds_b = (opt.precision == OPO_F64 ? lds_elems<double>(static_cast<int>(max_b))
                                         : lds_elems<float>(static_cast<int>(max_b))) * es;
    if (h->lds_a > 160 * 1024 || h->lds_b > 160 * 1024)
        return bail(fail(OPO_EINVAL, "internal: tile needs more LDS than a workgroup has"));

    // stage-major butterfly twiddles (fft_tile.h, tw_index)
    std::vector<double> twre(kTwEntries, 1.0), twim(kTwEntries, 0.0);
    for (int rs : {2, 4, 8, 16})
        for (int p = 1; p * rs <= kTwL; p *= 2)
            for (int k = 0; k < p; ++k)
                for (int r = 1; r < rs; ++r) {
                    const double a = kTwoPi * static_cast<double>(r * k) / static_cast<double>(p * rs);
                    twre[tw_index(rs, p, k) + r - 1] = std::cos(a);
                    twim[tw_index(rs, p, k) + r - 1] = -std::sin(a);
                }
    hipStream_t st = h->stream;
    if (hipMemcpyAsync(h->d_inst, h->inst.data(), h->inst.size() * sizeof(InstDesc), hipMemcpyHostToDevice, st) !=
            hipSuccess ||
        hipMemcpyAsync(h->d_tile_a, tile_a_inst.data(), tile_a_inst.size() * sizeof(int), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(h->d_tile_b, tile_b_inst.data(), tile_b_inst.size() * sizeof(int), hipMemcpyHostToDevice, st) != hipSuccess ||
        (h->mixed && hipMemcpyAsync(h->d_map[0], maps[0].data(), maps[0].size() * sizeof(int), hipMemcpyHostToDevice, st) != hipSuccess) ||
        (h->mixed && hipMemcpyAsync(h->d_map[1], maps[1].data(), maps[1].size() * sizeof(int), hipMemcpyHostToDevice, st) != hipSuccess) ||
        (!res_inst.empty() && hipMemcpyAsync(h->d_res_inst, res_inst.data(), res_inst.size() * sizeof(int),
                                             hipMemcpyHostToDevice, st) != hipSuccess) ||
        hipStreamSynchronize(st) != hipSuccess)
        return bail(fail(OPO_EDEVICE, "upload of the instance tables failed"));
    if ((opt.precision == OPO_F64 ? upload_phasors<double>(h->d_tw, twre, twim, st)
                                  : upload_phasors<float>(h->d_tw, twre, twim, st)) != hipSuccess)
        return bail(fail(OPO_EDEVICE, "upload of the FFT twiddles failed"));
    {
        // W_nt^{j1 k2} = e^{-2 pi i (j1 k2 mod nt)/nt} in FP64 at k2 * n1 + j1
        std::vector<double> wre(static_cast<size_t>(w4_elems)), wim(static_cast<size_t>(w4_elems));
        for (const auto &e : w4map) {
            const long long nt4 = 1LL << e.first.first, n1 = 1LL << e.first.second, n2 = nt4 / n1;
            for (long long k2 = 0; k2 < n2; ++k2)
                for (long long j1 = 0; j1 < n1; ++j1) {
                    const long long m = (j1 * k2) & (nt4 - 1);
                    const double a = kTwoPi * static_cast<double>(m) / static_cast<double>(nt4);
                    wre[e.second + k2 * n1 + j1] = std::cos(a);
                    wim[e.second + k2 * n1 + j1] = -std::sin(a);
                }
        }
        if ((opt.precision == OPO_F64 ? upload_phasors<double>(h->d_w4tab, wre, wim, st)
                                      : upload_phasors<float>(h->d_w4tab, wre, wim, st)) != hipSuccess)
            return bail(fail(OPO_EDEVICE, "upload of the four-step twiddles failed"));
    }
    std::vector<double> zeros;
    for (int i = 0; i < n; ++i) {
        const InstDesc &d = h->inst[i];
        const double *src = f[i].init;
        const long long count = static_cast<long long>(d.nf) * d.nt;
        if (!src) {
            zeros.assign(2 * static_cast<size_t>(count), 0.0);
            src = zeros.data();
        }
        char *dst = static_cast<char *>(h->state) + d.off * es;
        if ((opt.precision == OPO_F64 ? host_to_state<double>(dst, src, count, st)
                                      : host_to_state<float>(dst, src, count, st)) != hipSuccess)
            return bail(fail(OPO_EDEVICE, "upload of the initial fields failed"));
        if (f[i].pump_in) {
            char *pd = static_cast<char *>(h->pump) + d.pump_off * es;
            const long long count = static_cast<long long>(d.nt) * d.pump_windows;
            if ((opt.precision == OPO_F64 ? host_to_state<double>(pd, f[i].pump_in, count, st)
                                          : host_to_state<float>(pd, f[i].pump_in, count, st)) != hipSuccess)
                return bail(fail(OPO_EDEVICE, "upload of the input pump failed"));
        }
    }
    set_counter<<<1, 1, 0, st>>>(h->d_counter, 0, 0, 1);
    int krc = opt.precision == OPO_F64 ? setup_kernels<double>(h) : setup_kernels<float>(h);
    if (krc) return bail(krc);
    hipError_t le = hipGetLastError();
    if (le != hipSuccess) return bail(fail(OPO_EDEVICE, std::string("init: ") + hipGetErrorString(le)));
    for (int i = 0; i < n; ++i) h->t_window.push_back(f[i].t_window_ps);
    // output power of field x per unit beam area from its recorded energy E_x:
    // mean intensity n_x eps0 c E_x / (2 nt), times 1 - R_x through the output
    // coupler of a resonant field, or whole for a non-resonant one
    constexpr double kEps0 = 8.8541878128e-12, kC0 = 299792458.0;
    for (int i = 0; i < n; ++i)
        for (int x = 0; x < 3; ++x) {
            const bool used = x < nfields(f[i]);
            const double t = k[i].resonant[x] ? 1.0 - k[i].refl[x] : 1.0;
            h->out_scale.push_back(used ? t * 0.5 * f[i].n[x] * kEps0 * kC0 / f[i].nt : 0.0);
        }
    {
        std::lock_guard<std::mutex> lk(g_live_mu);
        g_live.insert(h);
    }
    *out = h;
    return OPO_OK;
}

static int check(opo_t *h)
{
    if (!is_live(h)) return fail(OPO_ESTATE, "invalid or destroyed handle");
    if (hipSetDevice(h->device) != hipSuccess) return fail(OPO_EDEVICE, "hipSetDevice failed");
    return OPO_OK;
}

// Fill the linear-propagator tables for a step dz (mode > 0) or for each
// instance's own L/nz (mode 0), unless they already hold that step.
template <typename R> static int ensure_tables(opo_t *h, double mode)
{
    if (h->disp_mode == mode) return OPO_OK;
    for (int o : h->disp_owner) {
        const InstDesc &d = h->inst[o];
        const double dz = mode > 0.0 ? mode : d.length_mm / h->stage_nz[o / h->n_inst];
        const int blocks = static_cast<int>(
            std::min<long long>((static_cast<long long>(d.nf) * d.nt + kThreads - 1) / kThreads, 4096));
        if (h->order == 4) {
            // propagators of the a dz and b dz steps of the composition
            disp_table<R><<<blocks, kThreads, 0, h->stream>>>(h->d_inst, o, static_cast<Phasor<R> *>(h->d_disp),
                                                              kTjA * dz, 0);
            disp_table<R><<<blocks, kThreads, 0, h->stream>>>(h->d_inst, o, static_cast<Phasor<R> *>(h->d_disp),
                                                              kTjB * dz, 1);
        } else {
            disp_table<R><<<blocks, kThreads, 0, h->stream>>>(h->d_inst, o, static_cast<Phasor<R> *>(h->d_disp),
                                                              dz, 0);
        }
    }
    HIP_TRY(hipGetLastError());
    h->disp_mode = mode;
    return OPO_OK;
}

template <typename R> static int propagate_impl(opo_t *h, int nz, double dz)
{
    int trc = ensure_tables<R>(h, dz);
    if (trc) return trc;
    StepArgs<R> a = base_args<R>(h, h->state);
    a.dz_arg = dz;
    a.zbase = h->z;
    {
        StepArgs<R> ar = a;
        ar.nz = nz;
        HIP_TRY(launch_resident<R>(h, ar, 0));
    }
    HIP_TRY(enqueue_pass<R>(h, a, nz, 0, 0));
    HIP_TRY(join_resident(h));
    h->z += nz * dz;
    const size_t used = h->ev_used;
    h->ev_used = 0;
    return prof_collect(h, used);
}

// Adaptive step: every instance from the handle's z over `length` (see
// adapt_control for the step control). Attempts are queued in chunks; the
// control state is read back after each chunk to see whether all have
// stopped.
// One attempt of the adaptive step for every running instance: begin, one
// step of dz on the coarse copy, two of dz/2 on the fine copy, the error
// sums and the control decision. Every launch argument is fixed once the
// buffers exist (z, dz, tol and the budget live in the control state), so
// the sequence is captured once into a graph and replayed.
template <typename R> static hipError_t enqueue_attempt(opo_t *h)
{
    const int blocks = h->a_chunks * h->n_inst;
    cplx<R> *u = static_cast<cplx<R> *>(h->state), *uc = static_cast<cplx<R> *>(h->a_uc),
            *uf = static_cast<cplx<R> *>(h->a_uf);
    Phasor<R> *tab = static_cast<Phasor<R> *>(h->a_tab);
    StepArgs<R> a = base_args<R>(h, h->a_uc);
    a.adapt = h->d_actl;
    a.disp = tab;
    adapt_begin<R><<<blocks, kThreads, 0, h->stream>>>(h->d_inst, h->d_actl, h->a_chunks, u, uc, uf, tab);
    HIP_RET(hipGetLastError());
    a.state = uc;                 // one step of dz, from u
    a.adapt_scale = 1.0;
    a.src = u;
    HIP_RET(launch_a<R>(h, a, A_RK_THIS | A_FWD, 0, -1, true));
    a.src = nullptr;
    HIP_RET(launch_b<R>(h, a, B_DISP, 0, 0, true));
    HIP_RET(launch_a<R>(h, a, A_INV | A_RK_PREV, 1, -1, true));
    a.state = uf;                 // two steps of dz/2, from u
    a.adapt_scale = 0.5;
    a.src = u;
    HIP_RET(launch_a<R>(h, a, A_RK_THIS | A_FWD, 0, -1, true));
    a.src = nullptr;
    HIP_RET(launch_b<R>(h, a, B_DISP, 0, 0, true));
    HIP_RET(launch_a<R>(h, a, A_INV | A_RK_PREV | A_RK_THIS | A_FWD, 1, -1, true));
    HIP_RET(launch_b<R>(h, a, B_DISP, 1, 0, true));
    HIP_RET(launch_a<R>(h, a, A_INV | A_RK_PREV, 2, -1, true));
    adapt_error<R><<<blocks, kThreads, 0, h->stream>>>(h->d_inst, h->d_actl, h->a_chunks, uc, uf, h->d_apart);
    HIP_RET(hipGetLastError());
    adapt_control<<<(h->n_inst + kThreads / 64 - 1) / (kThreads / 64), kThreads, 0, h->stream>>>(
        h->d_actl, h->n_inst, h->a_chunks, h->d_apart, 1, 0.0, 0.0, 0.0, 0.0, 0);
    return hipGetLastError();
}

// Adaptive step: every instance from the handle's z over `length` (see
// adapt_control for the step control). Attempts are queued in chunks sized
// by the remaining distance over the current step of the slowest instance;
// the control state is read back after each chunk to see whether all have
// stopped.
template <typename R>
static int adaptive_impl(opo_t *h, double length, double tol, double dz0, int max_attempts, int32_t *accepted,
                         int32_t *rejected, double *z_end)
{
    const size_t n_elem = h->state_bytes / h->elem;
    if (!h->a_uc) {
        long long max_n = 0;
        for (const InstDesc &d : h->inst)
            max_n = std::max(max_n, static_cast<long long>(d.nf) * d.nt);
        h->a_chunks = static_cast<int>(std::min<long long>((max_n + 8LL * kThreads - 1) / (8LL * kThreads), 256));
        if (static_cast<long long>(h->a_chunks) * h->n_inst > 2147483647LL)
            return fail(OPO_EINVAL, "too many instances for the adaptive step");
        if (hipMalloc(&h->a_uc, h->state_bytes) != hipSuccess || hipMalloc(&h->a_uf, h->state_bytes) != hipSuccess ||
            hipMalloc(&h->a_tab, n_elem * sizeof(Phasor<R>)) != hipSuccess ||
            hipMalloc(&h->d_actl, h->n_inst * sizeof(AdaptState)) != hipSuccess ||
            hipMalloc(&h->d_apart, 2 * sizeof(double) * h->a_chunks * h->n_inst) != hipSuccess) {
            // all or none: a later call allocates again
            void **bufs[] = {&h->a_uc, &h->a_uf, &h->a_tab, reinterpret_cast<void **>(&h->d_actl),
                             reinterpret_cast<void **>(&h->d_apart)};
            for (void **b : bufs) {
                if (*b) (void)hipFree(*b);
                *b = nullptr;
            }
            return fail(OPO_ENOMEM, "hipMalloc of the adaptive-step buffers failed");
        }
    }
    const int blocks = h->a_chunks * h->n_inst;
    if (h->use_graph && !h->a_graph) {
        hipGraph_t g;
        HIP_TRY(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
        const hipError_t qe = enqueue_attempt<R>(h);
        hipError_t ce = hipStreamEndCapture(h->stream, &g);
        if (qe != hipSuccess) {
            if (ce == hipSuccess) (void)hipGraphDestroy(g);
            return fail(OPO_EDEVICE, std::string("adaptive attempt: ") + hipGetErrorString(qe));
        }
        if (ce != hipSuccess) return fail(OPO_EDEVICE, std::string("graph capture: ") + hipGetErrorString(ce));
        ce = hipGraphInstantiate(&h->a_graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ce != hipSuccess) {
            h->a_graph = nullptr;
            return fail(OPO_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(ce));
        }
    }
    adapt_control<<<(h->n_inst + kThreads / 64 - 1) / (kThreads / 64), kThreads, 0, h->stream>>>(
        h->d_actl, h->n_inst, h->a_chunks, h->d_apart, 0, h->z, length, dz0, tol, max_attempts);
    HIP_TRY(hipGetLastError());
    std::vector<AdaptState> ctl(h->n_inst);
    HIP_TRY(hipMemcpyAsync(ctl.data(), h->d_actl, ctl.size() * sizeof(AdaptState), hipMemcpyDeviceToHost,
                           h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    for (;;) {
        // attempts the slowest running instance needs at least: its steps
        // growing by 2^(1/3) each time reach the end after n with
        // dz (g^n - 1)/(g - 1) >= rest (at least one, at most 64 per chunk)
        double need = 0.0;
        bool running = false;
        for (const AdaptState &st : ctl)
            if (st.status == 0) {
                running = true;
                const double n = std::log1p((st.end - st.z) * (kAdaptGrow - 1.0) / st.dz) / std::log(kAdaptGrow);
                need = std::max(need, std::ceil(n - 1e-9));
            }
        if (!running) break;
        const int chunk = static_cast<int>(std::min(std::max(need, 1.0), 64.0));
        for (int r = 0; r < chunk; ++r) {
            if (h->a_graph) {
                HIP_TRY(hipGraphLaunch(h->a_graph, h->stream));
            } else {
                HIP_TRY(enqueue_attempt<R>(h));
            }
        }
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(ctl.data(), h->d_actl, ctl.size() * sizeof(AdaptState), hipMemcpyDeviceToHost,
                               h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
        const size_t used = h->ev_used;
        h->ev_used = 0;
        int prc = prof_collect(h, used);
        if (prc) return prc;
    }
    // extrapolate the steps kept by the last attempts
    adapt_begin<R><<<blocks, kThreads, 0, h->stream>>>(h->d_inst, h->d_actl, h->a_chunks,
                                                       static_cast<cplx<R> *>(h->state), static_cast<cplx<R> *>(h->a_uc),
                                                       static_cast<cplx<R> *>(h->a_uf),
                                                       static_cast<Phasor<R> *>(h->a_tab));
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(h->stream));
    bool spent = false;
    for (int i = 0; i < h->n_inst; ++i) {
        if (accepted) accepted[i] = ctl[i].accepted;
        if (rejected) rejected[i] = ctl[i].rejected;
        if (z_end) z_end[i] = ctl[i].z;
        spent = spent || ctl[i].status == 2;
    }
    h->z += length;
    if (spent) return fail(OPO_ESTEPS, "adaptive step: attempt budget spent before the end");
    return OPO_OK;
}

// Round trips in chunks of up to kHistChunk graph replays, the energy rows of
// each chunk read back at its end. A round trip with non-finite energies (or
// a non-finite value stored at its end) sets the device stop flag: every later
// launch of the call stores nothing, the round trip's row is not counted, and
// the state is restored from the snapshot its refresh launch took, i.e. to the
// end of the last finite round trip.
template <typename R> static int roundtrip_impl(opo_t *h, int n_rt)
{
    int trc = ensure_tables<R>(h, 0.0);
    if (trc) return trc;
    if (h->use_graph && !h->graph) {
        hipGraph_t g;
        HIP_TRY(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
        const hipError_t qe = enqueue_roundtrip<R>(h);
        hipError_t ce = hipStreamEndCapture(h->stream, &g);
        if (qe != hipSuccess) {
            if (ce == hipSuccess) (void)hipGraphDestroy(g);
            return fail(OPO_EDEVICE, std::string("round trip: ") + hipGetErrorString(qe));
        }
        if (ce != hipSuccess) return fail(OPO_EDEVICE, std::string("graph capture: ") + hipGetErrorString(ce));
        ce = hipGraphInstantiate(&h->graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ce != hipSuccess) {
            h->graph = nullptr;
            return fail(OPO_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(ce));
        }
    }
    int done = 0;
    std::vector<double> chunk;
    int ctr[4] = {0, 0, 0, 0};
    while (done < n_rt) {
        const int m = std::min(kHistChunk, n_rt - done);
        set_counter<<<1, 1, 0, h->stream>>>(h->d_counter, 0, -1, 0);
        HIP_TRY(hipGetLastError());
        for (int r = 0; r < m; ++r) {
            if (h->graph) {
                HIP_TRY(hipGraphLaunch(h->graph, h->stream));
            } else {
                HIP_TRY(enqueue_roundtrip<R>(h));
                const size_t used = h->ev_used;
                h->ev_used = 0;
                int prc = prof_collect(h, used);
                if (prc) return prc;
            }
        }
        chunk.resize(static_cast<size_t>(m) * h->n_inst * 3);
        HIP_TRY(hipMemcpyAsync(chunk.data(), h->d_hist, chunk.size() * sizeof(double),
                               hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(hipMemcpyAsync(ctr, h->d_counter, sizeof(ctr), hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
        const int rows = std::min(ctr[0], m);   // finite round trips of this chunk
        h->hist.insert(h->hist.end(), chunk.begin(), chunk.begin() + static_cast<size_t>(rows) * h->n_inst * 3);
        h->hist_rows += rows;
        if (ctr[2] != 0) {
            // back to the end of the last finite round trip, flags cleared
            HIP_TRY(hipMemcpyAsync(h->state, h->d_snap, h->state_bytes, hipMemcpyDeviceToDevice, h->stream));
            set_counter<<<1, 1, 0, h->stream>>>(h->d_counter, 0, -1, 1);
            HIP_TRY(hipGetLastError());
            HIP_TRY(hipStreamSynchronize(h->stream));
            h->z = 0.0;
            return fail(OPO_ENONFINITE, "non-finite energy or field at round trip " + std::to_string(h->hist_rows) +
                                            " (counted from opo_init); stopped with the state that round trip "
                                            "started from");
        }
        done += m;
    }
    h->z = 0.0;
    return OPO_OK;
}

template <typename R> static int spectrum_impl(opo_t *h, int inst, int field, double *out)
{
    const InstDesc &d = h->inst[inst];
    if (!h->spec_buf) {
        if (hipMalloc(&h->spec_buf, h->state_bytes) != hipSuccess)
            return fail(OPO_ENOMEM, "hipMalloc of the spectrum buffer failed");
    }
    HIP_TRY(hipMemcpyAsync(h->spec_buf, h->state, h->state_bytes, hipMemcpyDeviceToDevice, h->stream));
    StepArgs<R> a = base_args<R>(h, h->spec_buf);
    HIP_TRY(launch_a<R>(h, a, A_FWD, 0, -1, true));
    HIP_TRY(launch_b<R>(h, a, B_FWD_ONLY, 0, -1, true));
    std::vector<double> tmp(2 * static_cast<size_t>(d.nt));
    const char *src = static_cast<const char *>(h->spec_buf) + (d.off + static_cast<long long>(field) * d.nt) * h->elem;
    HIP_TRY(state_to_host<R>(tmp.data(), src, d.nt, h->stream));
    // position k2*n1 + k1 holds bin k2 + n2*k1
    for (int k2 = 0; k2 < d.n2; ++k2)
        for (int k1 = 0; k1 < d.n1; ++k1) {
            const long long pos = static_cast<long long>(k2) * d.n1 + k1;
            const long long bin = k2 + static_cast<long long>(d.n2) * k1;
            out[2 * bin] = tmp[2 * pos];
            out[2 * bin + 1] = tmp[2 * pos + 1];
        }
    return OPO_OK;
}

// ---- spectrum read-out without allocation. Scratch lives in a fixed device
// array (each GPU the library runs on holds its own copy until the process
// ends): the descriptor of a one-instance batch, its tile -> instance map and
// counters, then the instance's fields as the column and row passes leave them.
// Calls on one GPU share the array: calls that overlap there race.
static constexpr size_t kNoAllocBytes = size_t(16) << 20;
static constexpr size_t kNoAllocCounterOff = 1024;     // 4 ints
static constexpr size_t kNoAllocMapOff = 2048;         // tile -> instance map
static constexpr size_t kNoAllocMapInts = 3584;
static constexpr size_t kNoAllocFieldOff = 16384;      // fields, 256-byte aligned
static_assert(sizeof(InstDesc) <= kNoAllocCounterOff, "descriptor does not fit its scratch slot");
static_assert(kNoAllocMapOff + kNoAllocMapInts * sizeof(int) <= kNoAllocFieldOff, "map overlaps the fields");

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

// Device address of `scratch` per device, taken once with that device current
// (in host code the array's name is only a stand-in for it).
static std::mutex g_scratch_mu;
static std::map<int, unsigned char *> g_scratch_ptr;

static int scratch_on_device(int device, unsigned char **out)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(device);
    if (it == g_scratch_ptr.end()) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr)
            return fail(OPO_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        it = g_scratch_ptr.emplace(device, static_cast<unsigned char *>(p)).first;
    }
    *out = it->second;
    return OPO_OK;
}

// The column pass (forward column FFT and four-step twiddle) loads instance
// `inst` from the state and stores into the scratch fields, the row pass
// finishes the forward transform in place, and spectrum_order writes natural
// bin order into `out`. The same kernels as the domain-1 read-out of
// opo_get_fields, on the same tiles, so the values are identical.
template <typename R> static int spectrum_noalloc_impl(opo_t *h, int inst, void *out)
{
    const InstDesc &d = h->inst[inst];
    const size_t field_bytes = static_cast<size_t>(d.nf) * static_cast<size_t>(d.nt) * sizeof(cplx<R>);
    const int map_len = std::max(d.tiles_a, d.tiles_b);
    if (field_bytes > kNoAllocBytes - kNoAllocFieldOff || static_cast<size_t>(map_len) > kNoAllocMapInts)
        return fail(OPO_EINVAL, "instance " + std::to_string(inst) + " needs " + std::to_string(field_bytes) +
                                    " bytes of scratch; the no-allocation read-out holds at most " +
                                    std::to_string(kNoAllocBytes - kNoAllocFieldOff));
    unsigned char *base = nullptr;
    int rc = scratch_on_device(h->device, &base);
    if (rc) return rc;
    InstDesc *desc = reinterpret_cast<InstDesc *>(base);
    int *counter = reinterpret_cast<int *>(base + kNoAllocCounterOff);
    int *map = reinterpret_cast<int *>(base + kNoAllocMapOff);
    cplx<R> *fields = reinterpret_cast<cplx<R> *>(base + kNoAllocFieldOff);

    spectrum_prep<<<1, kThreads, 0, h->stream>>>(h->d_inst, inst, desc, counter, map, map_len);
    HIP_TRY(hipGetLastError());
    StepArgs<R> a{};
    a.inst = desc;
    a.tile_inst = map;
    a.state = fields;
    a.src = static_cast<const cplx<R> *>(h->state) + d.off;
    a.tw = static_cast<const Phasor<R> *>(h->d_tw);
    a.w4tab = static_cast<const Phasor<R> *>(h->d_w4tab);
    a.disp = static_cast<const Phasor<R> *>(h->d_disp);
    a.counter = counter;
    a.nz = h->nz;
    a.flags = A_FWD;
    a.tile0 = 0;
    a.tile_count = d.tiles_a;
    {
        void *args[] = {&a};
        HIP_TRY(hipLaunchKernel(column_fn<R>(range_of(kColRanges, d.log2n2), d.nf), dim3(d.tiles_a),
                                dim3(kThreads), args, h->lds_a, h->stream));
    }
    a.src = nullptr;
    a.flags = B_FWD_ONLY;
    a.tile_count = d.tiles_b;
    {
        void *args[] = {&a};
        HIP_TRY(hipLaunchKernel(row_fn<R>(range_of(kRowRanges, d.log2n1)), dim3(d.tiles_b), dim3(kThreads), args,
                                h->lds_b, h->stream));
    }
    const long long n = static_cast<long long>(d.nf) * d.nt;
    const int blocks = static_cast<int>(std::min<long long>((n + kThreads - 1) / kThreads, 4096));
    spectrum_order<R><<<blocks, kThreads, 0, h->stream>>>(desc, fields, static_cast<cplx<R> *>(out));
    HIP_TRY(hipGetLastError());
    return OPO_OK;
}

} // namespace opo

extern "C" {

uint64_t opo_state_bytes(int32_t n, const opo_fields_t *fields, int32_t precision)
{
    if (n <= 0 || !fields) return 0;
    uint64_t s = 0;
    for (int i = 0; i < n; ++i)
        s += static_cast<uint64_t>(nfields(fields[i])) * static_cast<uint64_t>(fields[i].nt > 0 ? fields[i].nt : 0);
    return s * (precision == OPO_F64 ? 16 : 8);
}

int opo_init(opo_t **h, const opo_fields_t *fields, const opo_crystal_t *crystal,
             const opo_cavity_t *cavity, const opo_options_t *options)
{
    return opo_init_batch(h, 1, fields, crystal, cavity, options);
}

int opo_init_batch(opo_t **h, int32_t n, const opo_fields_t *fields, const opo_crystal_t *crystals,
                   const opo_cavity_t *cavities, const opo_options_t *options)
{
    if (!h) return fail(OPO_EINVAL, "handle pointer is NULL");
    *h = nullptr;
    if (n < 1 || !fields || !crystals || !cavities)
        return fail(OPO_EINVAL, "need n >= 1 and non-NULL fields, crystals and cavities");
    try {
        g_err.clear();
        return init_impl(h, n, fields, crystals, cavities, options);
    } catch (const std::bad_alloc &) {
        return fail(OPO_ENOMEM, "host allocation failed");
    } catch (...) {
        return fail(OPO_EDEVICE, "unexpected exception in opo_init");
    }
}

int ssfm_propagate(opo_t *h, int32_t nz, double dz)
{
    int rc = check(h);
    if (rc) return rc;
    if (nz < 1 || !(dz > 0.0) || !std::isfinite(dz)) return fail(OPO_EINVAL, "need nz >= 1 and finite dz > 0");
    try {
        return h->precision == OPO_F64 ? propagate_impl<double>(h, nz, dz) : propagate_impl<float>(h, nz, dz);
    } catch (...) {
        return fail(OPO_EDEVICE, "unexpected exception in ssfm_propagate");
    }
}

int ssfm_propagate_adaptive(opo_t *h, double length_mm, double tol, double dz0, int32_t max_attempts,
                            int32_t *accepted, int32_t *rejected, double *z_end)
{
    int rc = check(h);
    if (rc) return rc;
    if (!(length_mm >= 0.0) || !std::isfinite(length_mm) || !(tol > 0.0) || !std::isfinite(tol) ||
        !(dz0 > 0.0) || !std::isfinite(dz0) || max_attempts < 1)
        return fail(OPO_EINVAL, "need finite length_mm >= 0, tol > 0, dz0 > 0 and max_attempts >= 1");
    if (h->order != 2) return fail(OPO_EINVAL, "the adaptive step needs split_order 2");
    try {
        return h->precision == OPO_F64
                   ? adaptive_impl<double>(h, length_mm, tol, dz0, max_attempts, accepted, rejected, z_end)
                   : adaptive_impl<float>(h, length_mm, tol, dz0, max_attempts, accepted, rejected, z_end);
    } catch (...) {
        return fail(OPO_EDEVICE, "unexpected exception in ssfm_propagate_adaptive");
    }
}

int cavity_roundtrip(opo_t *h, int32_t n_rt)
{
    int rc = check(h);
    if (rc) return rc;
    if (n_rt < 0) return fail(OPO_EINVAL, "n_rt must be >= 0");
    try {
        return h->precision == OPO_F64 ? roundtrip_impl<double>(h, n_rt) : roundtrip_impl<float>(h, n_rt);
    } catch (const std::bad_alloc &) {
        return fail(OPO_ENOMEM, "host allocation failed");
    } catch (...) {
        return fail(OPO_EDEVICE, "unexpected exception in cavity_roundtrip");
    }
}

int opo_sync(opo_t *h)
{
    int rc = check(h);
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(h->stream));
    return OPO_OK;
}

int opo_get_fields(opo_t *h, int32_t inst, int32_t field, int32_t domain, double *out)
{
    int rc = check(h);
    if (rc) return rc;
    if (inst < 0 || inst >= h->n_inst || field < 0 || field >= h->inst[inst].nf || !out || domain < 0 ||
        domain > 1)
        return fail(OPO_EINVAL, "bad instance, field, domain or output pointer");
    try {
        if (domain == 1)
            return h->precision == OPO_F64 ? spectrum_impl<double>(h, inst, field, out)
                                           : spectrum_impl<float>(h, inst, field, out);
        const InstDesc &d = h->inst[inst];
        const char *src = static_cast<const char *>(h->state) + (d.off + static_cast<long long>(field) * d.nt) * h->elem;
        HIP_TRY(h->precision == OPO_F64 ? state_to_host<double>(out, src, d.nt, h->stream)
                                        : state_to_host<float>(out, src, d.nt, h->stream));
        return OPO_OK;
    } catch (...) {
        return fail(OPO_ENOMEM, "host allocation failed");
    }
}

int opo_set_fields(opo_t *h, int32_t inst, int32_t field, const double *in)
{
    int rc = check(h);
    if (rc) return rc;
    if (inst < 0 || inst >= h->n_inst || field < 0 || field >= h->inst[inst].nf || !in)
        return fail(OPO_EINVAL, "bad instance, field or input pointer");
    try {
        const InstDesc &d = h->inst[inst];
        char *dst = static_cast<char *>(h->state) + (d.off + static_cast<long long>(field) * d.nt) * h->elem;
        HIP_TRY(hipStreamSynchronize(h->stream));
        HIP_TRY(h->precision == OPO_F64 ? host_to_state<double>(dst, in, d.nt, h->stream)
                                        : host_to_state<float>(dst, in, d.nt, h->stream));
        h->z = 0.0;
        return OPO_OK;
    } catch (...) {
        return fail(OPO_ENOMEM, "host allocation failed");
    }
}

int opo_get_spectrum_noalloc(opo_t *h, int32_t inst, void *out)
{
    int rc = check(h);
    if (rc) return rc;
    if (inst < 0 || inst >= h->n_inst || !out) return fail(OPO_EINVAL, "bad instance or output pointer");
    try {
        return h->precision == OPO_F64 ? spectrum_noalloc_impl<double>(h, inst, out)
                                       : spectrum_noalloc_impl<float>(h, inst, out);
    } catch (...) {
        return fail(OPO_EDEVICE, "unexpected exception in opo_get_spectrum_noalloc");
    }
}

int opo_get_progress(opo_t *h, int32_t *rt_done, double *z_mm)
{
    int rc = check(h);
    if (rc) return rc;
    if (rt_done) *rt_done = h->hist_rows;
    if (z_mm) *z_mm = h->z;
    return OPO_OK;
}

int opo_set_progress(opo_t *h, int32_t rt_done, double z_mm, const double *history)
{
    int rc = check(h);
    if (rc) return rc;
    if (rt_done < 0 || (rt_done > 0 && !history) || !(z_mm >= 0.0) || !std::isfinite(z_mm))
        return fail(OPO_EINVAL, "need rt_done >= 0, a history for rt_done > 0, and finite z_mm >= 0");
    try {
        std::vector<double> hist(history, history + static_cast<size_t>(rt_done) * h->n_inst * 3);
        HIP_TRY(hipStreamSynchronize(h->stream));
        // the device count of completed round trips selects the input-pump window
        // and the record slot of the next one
        set_counter<<<1, 1, 0, h->stream>>>(h->d_counter, 0, rt_done, 1);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipStreamSynchronize(h->stream));
        h->hist.swap(hist);
        h->hist_rows = rt_done;
        h->z = z_mm;
        return OPO_OK;
    } catch (...) {
        return fail(OPO_ENOMEM, "host allocation failed");
    }
}

int opo_get_energy_history(opo_t *h, int32_t inst, double *out, int32_t capacity, int32_t *rows)
{
    int rc = check(h);
    if (rc) return rc;
    if (inst < 0 || inst >= h->n_inst || capacity < 0 || (capacity > 0 && !out))
        return fail(OPO_EINVAL, "bad instance, capacity or output pointer");
    const int m = std::min(capacity, h->hist_rows);
    for (int r = 0; r < m; ++r)
        for (int x = 0; x < 3; ++x)
            out[3 * r + x] = h->hist[(static_cast<size_t>(r) * h->n_inst + inst) * 3 + x];
    if (rows) *rows = h->hist_rows;
    return OPO_OK;
}

int opo_get_power_history(opo_t *h, int32_t inst, double area_m2, double *out, int32_t capacity, int32_t *rows)
{
    int rc = check(h);
    if (rc) return rc;
    if (inst < 0 || inst >= h->n_inst || capacity < 0 || (capacity > 0 && !out) || !(area_m2 > 0.0) ||
        !std::isfinite(area_m2))
        return fail(OPO_EINVAL, "bad instance, capacity, output pointer or area");
    const int m = std::min(capacity, h->hist_rows);
    for (int r = 0; r < m; ++r)
        for (int x = 0; x < 3; ++x)
            out[3 * r + x] = h->hist[(static_cast<size_t>(r) * h->n_inst + inst) * 3 + x] *
                             h->out_scale[3 * static_cast<size_t>(inst) + x] * area_m2;
    if (rows) *rows = h->hist_rows;
    return OPO_OK;
}

int opo_get_record(opo_t *h, int32_t inst, int32_t field, int32_t rt, double *out)
{
    int rc = check(h);
    if (rc) return rc;
    if (inst < 0 || inst >= h->n_inst || field < 0 || field >= h->inst[inst].nf || !out)
        return fail(OPO_EINVAL, "bad instance, field or output pointer");
    if (rt < 0 || rt >= std::min(h->record_cap, h->hist_rows))
        return fail(OPO_EINVAL, "round trip " + std::to_string(rt) + " is not in the record (capacity " +
                                    std::to_string(h->record_cap) + ", " + std::to_string(h->hist_rows) +
                                    " round trips run)");
    const InstDesc &d = h->inst[inst];
    const long long elems = static_cast<long long>(h->state_bytes / h->elem);
    const char *src = static_cast<const char *>(h->d_record) +
                      (static_cast<long long>(rt) * elems + d.off + static_cast<long long>(field) * d.nt) * h->elem;
    HIP_TRY(h->precision == OPO_F64 ? state_to_host<double>(out, src, d.nt, h->stream)
                                    : state_to_host<float>(out, src, d.nt, h->stream));
    return OPO_OK;
}

int opo_get_grid(opo_t *h, int32_t inst, double *t, double *omega)
{
    int rc = check(h);
    if (rc) return rc;
    if (inst < 0 || inst >= h->n_inst) return fail(OPO_EINVAL, "bad instance");
    const int nt = h->inst[inst].nt;
    const double T = h->t_window[inst];
    for (int j = 0; j < nt; ++j) {
        if (t) t[j] = -0.5 * T + j * (T / nt);
        if (omega) omega[j] = kTwoPi * (j < nt / 2 ? j : j - nt) / T;
    }
    return OPO_OK;
}

int opo_get_plan(opo_t *h, int32_t inst, int32_t *log2_n1, int32_t *log2_n2, int32_t *resident)
{
    int rc = check(h);
    if (rc) return rc;
    if (inst < 0 || inst >= h->n_inst) return fail(OPO_EINVAL, "bad instance");
    const InstDesc &d = h->inst[inst];
    if (log2_n1) *log2_n1 = d.log2n1;
    if (log2_n2) *log2_n2 = d.log2n2;
    if (resident) *resident = d.resident;
    return OPO_OK;
}

int opo_kernel_times(opo_t *h, double *ms, int64_t *launches)
{
    int rc = check(h);
    if (rc) return rc;
    for (int k = 0; k < OPO_K_CLASSES; ++k) {
        if (ms) ms[k] = h->k_ms[k];
        if (launches) launches[k] = h->k_count[k];
    }
    return OPO_OK;
}

int opo_info(opo_t *h, int32_t *n_instances, double *z_mm)
{
    int rc = check(h);
    if (rc) return rc;
    if (n_instances) *n_instances = h->n_inst;
    if (z_mm) *z_mm = h->z;
    return OPO_OK;
}

int opo_destroy(opo_t *h)
{
    if (!is_live(h)) return fail(OPO_ESTATE, "invalid or destroyed handle");
    release(h);
    return OPO_OK;
}

const char *opo_last_error(void) { return g_err.c_str(); }

} // extern "C"

// fsc_api.hip -- the C ABI of include/fsc.h: contexts, ensembles, graph
// replay, state transfer, measurement bookkeeping.  Host code only; all
// per-node work is done by the kernels of fsc_step.hip / fsc_measure.hip.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <map>
#include <memory>
#include <string>
#include <utility>
#include <vector>

#include "../../include/fsc.h"
#include "fsc_internal.h"

using namespace fsc;

namespace {

constexpr double CS2 = 1.0 / 3.0;

int q_of(int D) { return D == 2 ? 9 : 19; }

template <class L>
void lattice_tables(std::vector<int> &c, std::vector<double> &w, std::vector<double> &b,
                    std::vector<int> &cls) {
    c.resize(3 * L::Q);
    w.resize(L::Q);
    b.resize(L::Q);
    cls.resize(L::Q);
    for (int i = 0; i < L::Q; ++i) {
        for (int d = 0; d < 3; ++d) c[3 * i + d] = L::c(i, d);
        w[i] = L::w(i);
        b[i] = moment_norm<L>(i);
        cls[i] = L::cls(i);
    }
}

struct Rep {
    fsc_params p{};
    int Q = 0;
    int64_t N = 0;
    size_t esz = 4;
    void *buf[2] = {nullptr, nullptr};
    bool own = true;
    // lattice tables
    std::vector<int> c;
    std::vector<double> w, b;
    std::vector<int> cls;
    // structure factor
    int n_axis = 0, n_rad = 0;
    std::vector<int64_t> axis_modes, rad_modes;
    int64_t nsamples = 0;
    double *d_sk = nullptr;  // axis_sum, axis_sq, rad_sum, rad_sq
    void *cbuf = nullptr, *ctmp = nullptr;
    void *tw[3] = {nullptr, nullptr, nullptr};
    double *d_stats = nullptr, *d_partials = nullptr;
    // time series of samples: rows (step, L, per-shell mean S) -- see fsc_series_enable
    double *d_mom = nullptr, *d_series = nullptr;
    int *d_series_n = nullptr;
    int series_cap = 0;
    // recorded axis-mode amplitudes per sample -- see fsc_modes_enable
    double *d_modes = nullptr;
    int *d_modes_n = nullptr;
    int modes_nm = 0, modes_cap = 0;
    Geometry geom() const { return Geometry{p.D, p.nx, p.ny, p.nz, N}; }
};

// a population buffer of 4 GiB or more: beyond one 32-bit buffer resource
bool wide_buffer(const Rep &r) { return uint64_t(r.esz) * uint64_t(r.Q) * uint64_t(r.N) >= 0xffffffffull; }

struct GraphEntry {
    hipGraphExec_t exec = nullptr;
    int64_t samples = 0;
    int flips = 0;  // parity of the number of kernel launches (each swaps the buffers)
};

}  // namespace

struct fsc_ens {
    std::vector<Rep> reps;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int D = 2, stencil = 4, precision = 0;
    bool noise = false;
    TileShape tile{128, 1, 2};
    int64_t target_blocks = 2048;  // marching length is chosen to give about this many blocks
    int autotune = -1;             // -1: automatic for large lattices, 0: off, 1: done
    std::vector<RepDesc> desc;
    RepDesc *d_desc = nullptr;
    int *d_tile_begin = nullptr;
    uint64_t *d_step = nullptr;
    int64_t step = 0;
    int cur = 0;  // index of the buffer that holds the current state
    int total_tiles = 0;
    // batched S(k) sample of all replicas: host copy of the device table and its plan
    std::vector<MeasRep> meas;
    MeasPlan mplan;
    MeasRep *d_meas = nullptr;
    int *d_mpre = nullptr;
    std::string err;
    std::map<std::pair<int, std::pair<int64_t, int64_t>>, GraphEntry> graphs;
};

struct fsc_ctx {
    fsc_ens *e;
};

namespace {
thread_local std::string g_create_error;
}

namespace {

void ens_free(fsc_ens *e);

int fail(fsc_ens *e, int code, const std::string &msg) {
    if (e) e->err = msg;
    return code;
}

// Waits for the stream when a scope ends whose host buffers may still take
// part in an enqueued copy (an early return after a failed call).  Declared
// after those buffers, so that it runs before they are freed.
struct StreamDrain {
    hipStream_t s;
    ~StreamDrain() { (void)hipStreamSynchronize(s); }
};

#define HIPCHK(ens, expr)                                                            \
    do {                                                                             \
        hipError_t _e = (expr);                                                      \
        if (_e != hipSuccess)                                                        \
            return fail((ens), FSC_E_HIP,                                            \
                        std::string(#expr) + ": " + hipGetErrorString(_e));          \
    } while (0)

int resolve_params(const fsc_params &in, fsc_params &out, std::string &err) {
    out = in;
    if (in.D != 2 && in.D != 3) return err = "D must be 2 or 3", FSC_E_INVAL;
    if (in.nx < 1 || in.ny < 1 || in.nz < 1) return err = "sides must be >= 1", FSC_E_INVAL;
    if (in.D == 2 && in.nz != 1) return err = "nz must be 1 in 2D", FSC_E_INVAL;
    if (in.stencil != FSC_E4 && in.stencil != FSC_E8) return err = "stencil must be 4 or 8", FSC_E_INVAL;
    if (in.D == 3 && in.stencil == FSC_E8) return err = "E8 is 2D only", FSC_E_NOTSUP;
    if (in.precision != FSC_FP32_SHIFTED && in.precision != FSC_FP64)
        return err = "bad precision", FSC_E_INVAL;
    if (!(in.rho0 > 0.0) || !std::isfinite(in.rho0)) return err = "rho0 must be > 0", FSC_E_INVAL;
    const double lams[3] = {in.lambda_bulk, in.lambda_shear, in.lambda_ghost};
    for (double l : lams)
        if (!(l > 0.0 && l < 2.0)) return err = "relaxation rates must lie in (0, 2)", FSC_E_INVAL;
    if (!(in.kBT >= 0.0) || !std::isfinite(in.kBT)) return err = "kBT must be >= 0", FSC_E_INVAL;
    if (std::isnan(in.G)) {
        if (!(in.T_hat > 0.0) || !std::isfinite(in.T_hat))
            return err = "T_hat must be > 0 when G is NaN", FSC_E_INVAL;
        // critical point of p = nT - (G/2) exp(-2/n): T_c = G/e^2; T = 1/3
        out.G = std::exp(2.0) * CS2 / in.T_hat;
    } else {
        if (!std::isfinite(in.G)) return err = "G must be finite", FSC_E_INVAL;
        out.T_hat = in.G != 0.0 ? std::exp(2.0) * CS2 / in.G : INFINITY;
    }
    const int64_t N = int64_t(in.nx) * in.ny * in.nz;
    // the step kernels address one population (N values) with 32-bit byte
    // offsets; buffers of 4 GiB or more take one buffer resource per population
    const int64_t esz = in.precision == FSC_FP64 ? 8 : 4;
    if (N * esz >= (int64_t(1) << 32) - 1)
        return err = "lattice too large (one population must stay below 4 GiB)", FSC_E_INVAL;
    return FSC_OK;
}

int init_rep(Rep &r, const fsc_params &p, void *ext_a, void *ext_b, fsc_ens *e) {
    r.p = p;
    r.Q = q_of(p.D);
    r.N = int64_t(p.nx) * p.ny * p.nz;
    r.esz = p.precision == FSC_FP32_SHIFTED ? 4 : 8;
    if (p.D == 2) lattice_tables<D2Q9>(r.c, r.w, r.b, r.cls);
    else lattice_tables<D3Q19>(r.c, r.w, r.b, r.cls);
    const size_t bytes = r.esz * size_t(r.Q) * size_t(r.N);
    if (ext_a || ext_b) {
        if (!ext_a || !ext_b || ext_a == ext_b) return fail(e, FSC_E_INVAL, "need two distinct buffers");
        r.buf[0] = ext_a;
        r.buf[1] = ext_b;
        r.own = false;
    } else {
        for (int k = 0; k < 2; ++k)
            if (hipMalloc(&r.buf[k], bytes) != hipSuccess) {
                (void)hipGetLastError();
                return fail(e, FSC_E_OOM, "population buffer allocation failed");
            }
    }
    // S(k) geometry: modes per bin, exact integer rounding of |m|
    const int D = p.D;
    const int nmax = std::max(p.nx, std::max(p.ny, p.nz));
    r.n_axis = nmax / 2 + 1;
    const bool cubic = p.nx == p.ny && (D == 2 || p.ny == p.nz);
    auto round_sqrt = [](int64_t m) {
        int64_t b = int64_t(std::sqrt(double(m)));
        while (b * b > m) --b;
        while ((b + 1) * (b + 1) <= m) ++b;
        if (m - b * b > b) ++b;
        return int(b);
    };
    r.n_rad = cubic ? round_sqrt(int64_t(D) * (p.nx / 2) * (p.nx / 2)) + 1 : 0;
    r.axis_modes.assign(size_t(D) * r.n_axis, 0);
    r.rad_modes.assign(size_t(r.n_rad), 0);
    const int sides[3] = {p.nx, p.ny, p.nz};
    for (int d = 0; d < D; ++d)
        for (int q = 1; q < sides[d]; ++q) {
            const int m = q <= sides[d] / 2 ? q : sides[d] - q;
            r.axis_modes[size_t(d) * r.n_axis + m] += 1;
        }
    if (cubic) {
        const int L = p.nx;
        std::vector<int64_t> sq(L);
        for (int q = 0; q < L; ++q) {
            const int64_t m = q <= L / 2 ? q : q - L;
            sq[q] = m * m;
        }
        const int zmax = D == 3 ? L : 1;
        for (int z = 0; z < zmax; ++z)
            for (int y = 0; y < L; ++y)
                for (int x = 0; x < L; ++x) {
                    const int64_t m2 = sq[x] + sq[y] + (D == 3 ? sq[z] : 0);
                    if (m2) r.rad_modes[round_sqrt(m2)] += 1;
                }
    }
    const size_t nsk = 2 * size_t(D) * r.n_axis + 2 * size_t(r.n_rad);
    if (hipMalloc(&r.d_sk, sizeof(double) * nsk) != hipSuccess ||
        hipMalloc(&r.d_mom, sizeof(double) * 2) != hipSuccess ||
        hipMalloc(&r.d_series_n, sizeof(int)) != hipSuccess ||
        hipMalloc(&r.d_stats, sizeof(double) * 8) != hipSuccess ||
        hipMalloc(&r.d_partials, sizeof(double) * stats_partials_len()) != hipSuccess) {
        (void)hipGetLastError();
        return fail(e, FSC_E_OOM, "accumulator allocation failed");
    }
    HIPCHK(e, hipMemsetAsync(r.d_sk, 0, sizeof(double) * nsk, e->stream));
    HIPCHK(e, hipMemsetAsync(r.d_mom, 0, sizeof(double) * 2, e->stream));
    HIPCHK(e, hipMemsetAsync(r.d_series_n, 0, sizeof(int), e->stream));
    return FSC_OK;
}

// Buffers of the S(k) sample: complex field, scratch and twiddle tables.  The
// set counts as ready only when every part exists, so that a call that failed
// half way is completed (or fails again) on the next request.
int ensure_fft(Rep &r, fsc_ens *e) {
    const int sides[3] = {r.p.nx, r.p.ny, r.p.nz};
    bool ready = r.cbuf && r.ctmp;
    for (int d = 0; d < r.p.D; ++d) ready = ready && r.tw[d];
    if (ready) return FSC_OK;
    for (int d = 0; d < r.p.D; ++d)
        if (sides[d] > 8192) return fail(e, FSC_E_NOTSUP, "S(k) needs sides <= 8192");
    const size_t csz = 2 * r.esz * size_t(r.N);
    if ((!r.cbuf && hipMalloc(&r.cbuf, csz) != hipSuccess) ||
        (!r.ctmp && hipMalloc(&r.ctmp, csz) != hipSuccess)) {
        (void)hipGetLastError();
        return fail(e, FSC_E_OOM, "FFT buffer allocation failed");
    }
    for (int d = 0; d < r.p.D; ++d) {
        if (r.tw[d]) continue;
        void *tw = nullptr;
        if (hipMalloc(&tw, 2 * r.esz * twiddle_len(sides[d])) != hipSuccess) {
            (void)hipGetLastError();
            return fail(e, FSC_E_OOM, "twiddle allocation failed");
        }
        const hipError_t ec = launch_twiddles(r.p.precision, tw, sides[d], e->stream);
        if (ec != hipSuccess) {
            (void)hipFree(tw);
            return fail(e, FSC_E_HIP, std::string("twiddles: ") + hipGetErrorString(ec));
        }
        r.tw[d] = tw;
    }
    return FSC_OK;
}

// The device table of the batched S(k) sample is rebuilt from the replicas'
// current buffers before any sample is enqueued (outside graph capture).  When
// it changes (first use, series or mode recorder switched on or resized) the
// stream is drained, the table uploaded and the captured graphs dropped, since
// their launch sizes come from it.  Needs ensure_fft on every replica.
void drop_graphs(fsc_ens *e);

int ensure_measure_plan(fsc_ens *e) {
    const int n = int(e->reps.size());
    std::vector<MeasRep> m(static_cast<size_t>(n));
    for (int k = 0; k < n; ++k) {
        const Rep &r = e->reps[k];
        MeasRep &x = m[size_t(k)];
        std::memset(&x, 0, sizeof(MeasRep));
        if (!r.cbuf) return fail(e, FSC_E_STATE, "S(k) buffers missing");
        x.buf[0] = r.buf[0];
        x.buf[1] = r.buf[1];
        x.cbuf = r.cbuf;
        x.ctmp = r.ctmp;
        for (int d = 0; d < 3; ++d) x.tw[d] = r.tw[d];
        x.g = r.geom();
        const size_t na = size_t(r.p.D) * r.n_axis;
        x.t.axis_sum = r.d_sk;
        x.t.axis_sq = r.d_sk + na;
        x.t.rad_sum = r.n_rad ? r.d_sk + 2 * na : nullptr;
        x.t.rad_sq = r.n_rad ? r.d_sk + 2 * na + r.n_rad : nullptr;
        x.t.n_axis = r.n_axis;
        x.t.n_rad = r.n_rad;
        const bool ser = r.series_cap > 0;
        x.t.mom = ser ? r.d_mom : nullptr;
        x.t.series = ser ? r.d_series : nullptr;
        x.t.series_n = r.d_series_n;
        x.t.series_cap = r.series_cap;
        x.series_n = r.d_series_n;
        x.invN = 1.0 / double(r.N);
        if (r.modes_cap > 0) {
            x.modes = r.d_modes;
            x.modes_n = r.d_modes_n;
            x.modes_nm = r.modes_nm;
            x.modes_cap = r.modes_cap;
        }
    }
    if (e->d_meas && m.size() == e->meas.size() &&
        std::memcmp(m.data(), e->meas.data(), sizeof(MeasRep) * m.size()) == 0)
        return FSC_OK;
    MeasPlan P;
    P.esz = e->reps[0].esz;
    if (measure_plan(m.data(), n, P)) return fail(e, FSC_E_NOTSUP, "S(k) sample sizes out of range");
    HIPCHK(e, hipStreamSynchronize(e->stream));
    if (!e->d_meas) {
        if (hipMalloc(&e->d_meas, sizeof(MeasRep) * size_t(n)) != hipSuccess ||
            hipMalloc(&e->d_mpre, sizeof(int) * P.pre.size()) != hipSuccess) {
            (void)hipGetLastError();
            return fail(e, FSC_E_OOM, "S(k) table allocation failed");
        }
    }
    drop_graphs(e);
    HIPCHK(e, hipMemcpy(e->d_meas, m.data(), sizeof(MeasRep) * size_t(n), hipMemcpyHostToDevice));
    HIPCHK(e, hipMemcpy(e->d_mpre, P.pre.data(), sizeof(int) * P.pre.size(), hipMemcpyHostToDevice));
    e->meas = std::move(m);
    e->mplan = std::move(P);
    return FSC_OK;
}

// enqueues one S(k) sample of every replica from buffer `par`; the sampled
// state is `step_off` steps past the device step counter
int enqueue_measure(fsc_ens *e, int par, uint32_t step_off) {
    HIPCHK(e, launch_measure(e->mplan, e->d_meas, e->d_mpre, e->precision, par, e->d_step, step_off,
                             e->stream));
    return FSC_OK;
}

int modes_enable(fsc_ens *e, Rep &r, int nm, int cap) {
    (void)hipStreamSynchronize(e->stream);
    if (r.d_modes) {
        (void)hipFree(r.d_modes);
        r.d_modes = nullptr;
    }
    r.modes_cap = 0;
    r.modes_nm = 0;
    if (!r.d_modes_n) {
        if (hipMalloc(&r.d_modes_n, sizeof(int)) != hipSuccess) {
            (void)hipGetLastError();
            return fail(e, FSC_E_OOM, "mode recorder allocation failed");
        }
    }
    if (cap > 0) {
        const int sides[3] = {r.p.nx, r.p.ny, r.p.nz};
        for (int d = 0; d < r.p.D; ++d)
            if (nm > sides[d] / 2) return fail(e, FSC_E_INVAL, "nm exceeds half a side");
        const size_t bytes = sizeof(double) * 2 * size_t(cap) * size_t(r.p.D) * size_t(nm);
        if (hipMalloc(&r.d_modes, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return fail(e, FSC_E_OOM, "mode recorder allocation failed");
        }
        HIPCHK(e, hipMemsetAsync(r.d_modes, 0, bytes, e->stream));
        r.modes_cap = cap;
        r.modes_nm = nm;
    }
    HIPCHK(e, hipMemsetAsync(r.d_modes_n, 0, sizeof(int), e->stream));
    HIPCHK(e, hipStreamSynchronize(e->stream));
    return FSC_OK;
}

int modes_read(fsc_ens *e, Rep &r, double *out, int max_rows, int *nrows) {
    int n = 0;
    if (r.d_modes_n) {
        HIPCHK(e, hipMemcpyAsync(&n, r.d_modes_n, sizeof(int), hipMemcpyDeviceToHost, e->stream));
        HIPCHK(e, hipStreamSynchronize(e->stream));
    }
    n = std::min(n, r.modes_cap);
    const int m = std::min(n, max_rows);
    if (m > 0 && out) {
        HIPCHK(e, hipMemcpyAsync(out, r.d_modes, sizeof(double) * 2 * size_t(m) * r.p.D * r.modes_nm,
                                 hipMemcpyDeviceToHost, e->stream));
        HIPCHK(e, hipStreamSynchronize(e->stream));
    }
    if (nrows) *nrows = n;
    return FSC_OK;
}

int series_enable(fsc_ens *e, Rep &r, int cap) {
    (void)hipStreamSynchronize(e->stream);
    if (r.d_series) {
        (void)hipFree(r.d_series);
        r.d_series = nullptr;
    }
    r.series_cap = 0;
    if (cap > 0) {
        const size_t bytes = sizeof(double) * size_t(cap) * size_t(2 + r.n_rad);
        if (hipMalloc(&r.d_series, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return fail(e, FSC_E_OOM, "series allocation failed");
        }
        HIPCHK(e, hipMemsetAsync(r.d_series, 0, bytes, e->stream));
        r.series_cap = cap;
    }
    HIPCHK(e, hipMemsetAsync(r.d_series_n, 0, sizeof(int), e->stream));
    HIPCHK(e, hipMemsetAsync(r.d_mom, 0, sizeof(double) * 2, e->stream));
    HIPCHK(e, hipStreamSynchronize(e->stream));
    return FSC_OK;
}

int series_read(fsc_ens *e, Rep &r, double *out, int max_rows, int *nrows, int *row_len) {
    const int len = 2 + r.n_rad;
    if (row_len) *row_len = len;
    int n = 0;
    HIPCHK(e, hipMemcpyAsync(&n, r.d_series_n, sizeof(int), hipMemcpyDeviceToHost, e->stream));
    HIPCHK(e, hipStreamSynchronize(e->stream));
    n = std::min(n, r.series_cap);
    if (nrows) *nrows = n;
    if (!out || max_rows <= 0 || n == 0) return FSC_OK;
    const int m = std::min(n, max_rows);
    HIPCHK(e, hipMemcpyAsync(out, r.d_series, sizeof(double) * size_t(m) * len,
                             hipMemcpyDeviceToHost, e->stream));
    HIPCHK(e, hipStreamSynchronize(e->stream));
    for (int row = 0; row < m; ++row)
        for (int b = 0; b < r.n_rad; ++b)
            out[size_t(row) * len + 2 + b] =
                r.rad_modes[b] ? out[size_t(row) * len + 2 + b] / double(r.rad_modes[b]) : 0.0;
    if (nrows) *nrows = m;
    return FSC_OK;
}

// -------------------------------------------------------------------------
// Tiling of the fused step.
// -------------------------------------------------------------------------
void build_desc(fsc_ens *e) {
    e->desc.clear();
    int64_t work = 0;  // cross tiles x planes over the ensemble
    for (auto &r : e->reps) {
        const int tx = (r.p.nx + e->tile.tx - 1) / e->tile.tx;
        const int ty = r.p.D == 3 ? (r.p.ny + e->tile.ty - 1) / e->tile.ty : 1;
        const int ns = r.p.D == 3 ? r.p.nz : r.p.ny;
        work += int64_t(tx) * ty * ns;
    }
    // marching length: the shortest that gives at most target_blocks
    // workgroups (so that a target equal to the number resident at once
    // leaves no partial second round; each replica's chunks are then evened
    // out, which can only shorten them); long marches keep the halo planes a
    // small overhead
    auto blocks_for = [&](int h) {
        int64_t n = 0;
        for (auto &r : e->reps) {
            const int tx = (r.p.nx + e->tile.tx - 1) / e->tile.tx;
            const int ty = r.p.D == 3 ? (r.p.ny + e->tile.ty - 1) / e->tile.ty : 1;
            const int ns = r.p.D == 3 ? r.p.nz : r.p.ny;
            const int hh = std::min(h, ns);
            n += int64_t(tx) * ty * ((ns + hh - 1) / hh);
        }
        return n;
    };
    int H = int(std::min<int64_t>(256, std::max<int64_t>(1, (work + e->target_blocks - 1) / e->target_blocks)));
    while (H < 256 && blocks_for(H) > e->target_blocks) ++H;
    int tile_begin = 0;
    for (auto &r : e->reps) {
        RepDesc d{};
        d.buf[0] = r.buf[0];
        d.buf[1] = r.buf[1];
        d.N = r.N;
        d.nx = r.p.nx;
        d.ny = r.p.ny;
        d.nz = r.p.nz;
        d.ns = r.p.D == 3 ? r.p.nz : r.p.ny;
        d.plane = r.p.D == 3 ? r.p.nx * r.p.ny : r.p.nx;
        d.tiles_x = (r.p.nx + e->tile.tx - 1) / e->tile.tx;
        d.tiles_y = r.p.D == 3 ? (r.p.ny + e->tile.ty - 1) / e->tile.ty : 1;
        const int h = std::min(H, d.ns);
        const int nch = (d.ns + h - 1) / h;
        d.H = (d.ns + nch - 1) / nch;            // balanced chunk length
        d.nchunk = (d.ns + d.H - 1) / d.H;       // no empty trailing chunk
        d.tile_begin = tile_begin;
        tile_begin += d.tiles_x * d.tiles_y * d.nchunk;
        d.noise = r.p.kBT > 0.0;
        d.G = r.p.G;
        d.rho0 = r.p.rho0;
        d.psi0 = std::exp(-1.0 / r.p.rho0);
        const double lams[4] = {1.0, r.p.lambda_bulk, r.p.lambda_shear, r.p.lambda_ghost};
        for (int k = 0; k < 4; ++k) {
            const double g = 1.0 - lams[k];
            d.lamc[k] = lams[k];
            d.ampc[k] = k == 0 ? 0.0 : std::sqrt(r.p.kBT / CS2 * (1.0 - g * g));
            d.lamcf[k] = float(d.lamc[k]);
            d.ampcf[k] = float(d.ampc[k]);
        }
        d.Gf = float(d.G);
        d.rho0f = float(d.rho0);
        d.psi0f = float(d.psi0);
        d.inv_rho0f = float(1.0 / d.rho0);
        d.key0 = uint32_t(r.p.seed & 0xffffffffu);
        d.key1 = r.p.replica;
        d.seed_hi = uint32_t(r.p.seed >> 32);
        e->desc.push_back(d);
    }
    e->total_tiles = tile_begin;
}

int upload_desc(fsc_ens *e) {
    build_desc(e);
    const size_t n = e->desc.size();
    if (!e->d_desc) {
        if (hipMalloc(&e->d_desc, sizeof(RepDesc) * n) != hipSuccess ||
            hipMalloc(&e->d_tile_begin, sizeof(int) * n) != hipSuccess ||
            hipMalloc(&e->d_step, sizeof(uint64_t)) != hipSuccess) {
            (void)hipGetLastError();
            return fail(e, FSC_E_OOM, "descriptor allocation failed");
        }
    }
    std::vector<int> tb(n);
    for (size_t k = 0; k < n; ++k) tb[k] = e->desc[k].tile_begin;
    StreamDrain drain{e->stream};
    HIPCHK(e, hipMemcpyAsync(e->d_desc, e->desc.data(), sizeof(RepDesc) * n, hipMemcpyHostToDevice,
                             e->stream));
    HIPCHK(e, hipMemcpyAsync(e->d_tile_begin, tb.data(), sizeof(int) * n, hipMemcpyHostToDevice,
                             e->stream));
    HIPCHK(e, hipStreamSynchronize(e->stream));
    return FSC_OK;
}

int set_step_device(fsc_ens *e, int64_t step) {
    const uint64_t s = uint64_t(step);
    HIPCHK(e, hipMemcpyAsync(e->d_step, &s, sizeof(s), hipMemcpyHostToDevice, e->stream));
    HIPCHK(e, hipStreamSynchronize(e->stream));
    e->step = step;
    return FSC_OK;
}

void drop_graphs(fsc_ens *e) {
    for (auto &kv : e->graphs)
        if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
    e->graphs.clear();
}

StepLaunch make_launch(fsc_ens *e, int parity, uint32_t off) {
    StepLaunch L;
    L.reps = e->d_desc;
    L.tile_begin = e->d_tile_begin;
    L.nrep = int(e->reps.size());
    L.total_tiles = e->total_tiles;
    L.parity = parity;
    L.step_base = e->d_step;
    L.step_off = off;
    L.D = e->D;
    L.stencil = e->stencil;
    L.precision = e->precision;
    L.noise = e->noise;
    L.wide = false;
    for (const auto &r : e->reps) L.wide = L.wide || wide_buffer(r);
    L.tile = e->tile;
    return L;
}

// Enqueues n steps from buffer `cur`: with a two-step tiling, steps go in
// pairs except where an S(k) sample falls between them (and a last odd one);
// those run the single-step kernel of the same tile width, which uses the
// same tile table.  Returns the parity of the number of launches in *flips.
bool pair_from(const fsc_ens *e, int64_t k, int64_t n, int64_t sk_every) {
    return e->tile.steps == 2 && k + 1 < n && !(sk_every > 0 && (k + 1) % sk_every == 0);
}

// number of kernel launches enqueue_steps makes for n steps
int64_t count_launches(const fsc_ens *e, int64_t n, int64_t sk_every) {
    int64_t m = 0;
    for (int64_t k = 0; k < n; k += pair_from(e, k, n, sk_every) ? 2 : 1) ++m;
    return m;
}

int enqueue_steps(fsc_ens *e, int cur, int64_t n, int64_t sk_every, int64_t *samples, int *flips) {
    int c = cur, launches = 0;
    for (int64_t k = 0; k < n;) {
        const bool two = pair_from(e, k, n, sk_every);
        StepLaunch L = make_launch(e, c, uint32_t(k));
        if (!two && L.tile.steps == 2) L.tile = TileShape{L.tile.tx, 1, 1};
        HIPCHK(e, launch_step(L, e->stream));
        c ^= 1;
        ++launches;
        k += two ? 2 : 1;
        if (sk_every > 0 && k % sk_every == 0) {
            int rc = enqueue_measure(e, c, uint32_t(k));
            if (rc) return rc;
            if (samples) ++*samples;
        }
    }
    HIPCHK(e, launch_step_advance(e->d_step, uint64_t(n), e->stream));
    if (flips) *flips = launches & 1;
    return FSC_OK;
}

// Two-step tilings need 2D FP32 lattices at least 2R + 2 columns wide.
// the two-step kernel addresses a whole buffer with 32-bit offsets, and needs
// 2R + 2 columns
bool two_step_ok(const fsc_ens *e) {
    if (e->D != 2 || e->precision != FSC_FP32_SHIFTED) return false;
    const int R = e->stencil == FSC_E8 ? 2 : 1;
    for (const auto &r : e->reps)
        if (r.p.nx < 2 * R + 2 || wide_buffer(r)) return false;
    return true;
}

// -------------------------------------------------------------------------
// Autotuner: times every compiled tile shape and marching-length target on the
// ensemble's own buffers and keeps the fastest.  Trial launches alternate
// between the two buffers as a run does (each reads what the one before
// wrote); the state is copied aside first and put back afterwards, and the
// step counter is not advanced, so tuning leaves the state untouched.  Without
// room for the copy every trial launch reads the current buffer and writes the
// other, which holds nothing needed (that times the caches differently from a
// run and can prefer a slower march length).  The per-node arithmetic does not
// depend on the tiling, so neither do results.
// -------------------------------------------------------------------------
struct TuneChoice {
    TileShape tile;
    int64_t target;
};
std::mutex g_tune_mu;
std::map<std::string, TuneChoice> g_tune_cache;

std::string tune_key(const fsc_ens *e) {
    std::string k = std::to_string(e->D) + "/" + std::to_string(e->stencil) + "/" +
                    std::to_string(e->precision) + "/" + std::to_string(int(e->noise));
    for (const auto &r : e->reps)
        k += ":" + std::to_string(r.p.nx) + "x" + std::to_string(r.p.ny) + "x" + std::to_string(r.p.nz);
    return k;
}

int ens_autotune(fsc_ens *e) {
    TraceRange trace_("fsc autotune");
    const std::string key = tune_key(e);
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            e->tile = it->second.tile;
            e->target_blocks = it->second.target;
            drop_graphs(e);
            e->autotune = 1;
            return upload_desc(e);
        }
    }
    TileShape shapes[32];
    const int nshape = tile_shapes(e->D, e->stencil, e->precision, shapes, 32);
    // block counts of one round of resident workgroups (a multiple of the
    // 256 CUs: 1-8 per CU, depending on the kernel's LDS and registers) and
    // of several rounds
    const int64_t targets[] = {256,  512,  768,  1024, 1280, 1536, 1792,  2048,  2304,
                               2560, 3072, 3584, 4096, 4608, 6144, 8192, 12288, 16384};
    hipEvent_t a, b;
    HIPCHK(e, hipEventCreate(&a));
    HIPCHK(e, hipEventCreate(&b));
    TuneChoice choice{e->tile, e->target_blocks};
    const int parity = e->cur;
    // the state, copied aside for the alternating trials and put back on every
    // way out of this function
    struct StateCopy {
        fsc_ens *e;
        int parity;
        std::vector<void *> saved;
        static size_t bytes(const Rep &r) { return size_t(r.Q) * size_t(r.N) * r.esz; }
        ~StateCopy() {
            for (size_t i = 0; i < saved.size(); ++i)
                (void)hipMemcpyAsync(e->reps[i].buf[parity], saved[i], bytes(e->reps[i]),
                                     hipMemcpyDeviceToDevice, e->stream);
            if (!saved.empty()) (void)hipStreamSynchronize(e->stream);
            for (void *q : saved) (void)hipFree(q);
        }
    } copy{e, parity, {}};
    bool alternate = true;
    for (const Rep &r : e->reps) {
        void *q = nullptr;
        if (hipMalloc(&q, StateCopy::bytes(r)) != hipSuccess) {
            (void)hipGetLastError();
            alternate = false;
            break;
        }
        const hipError_t ce = hipMemcpyAsync(q, r.buf[parity], StateCopy::bytes(r), hipMemcpyDeviceToDevice, e->stream);
        if (ce != hipSuccess) {  // only complete copies are put back
            (void)hipFree(q);
            return fail(e, FSC_E_HIP, std::string("autotune state copy: ") + hipGetErrorString(ce));
        }
        copy.saved.push_back(q);
    }
    if (!alternate) {
        HIPCHK(e, hipStreamSynchronize(e->stream));
        for (void *q : copy.saved) (void)hipFree(q);
        copy.saved.clear();
    }
    // the fastest of `windows` windows of `per` launches, per step (robust to
    // a transient slowdown of one window)
    auto time_choice = [&](const TuneChoice &c, int windows, int per, float *ms_out) -> int {
        e->tile = c.tile;
        e->target_blocks = c.target;
        int rc = upload_desc(e);
        if (rc) return rc;
        const StepLaunch L[2] = {make_launch(e, parity, 0), make_launch(e, alternate ? parity ^ 1 : parity, 0)};
        int n = 0;  // launches so far: buffer parity of the next one
        for (int k = 0; k < 2; ++k) HIPCHK(e, launch_step(L[n++ & 1], e->stream));
        float ms = 1e30f;
        for (int w = 0; w < windows; ++w) {
            HIPCHK(e, hipEventRecord(a, e->stream));
            for (int k = 0; k < per; ++k) HIPCHK(e, launch_step(L[n++ & 1], e->stream));
            HIPCHK(e, hipEventRecord(b, e->stream));
            HIPCHK(e, hipEventSynchronize(b));
            float t = 0.f;
            HIPCHK(e, hipEventElapsedTime(&t, a, b));
            ms = std::min(ms, t);
        }
        *ms_out = ms / float(per * c.tile.steps);
        return FSC_OK;
    };
    std::vector<std::pair<float, TuneChoice>> timed;
    for (int si = 0; si < nshape; ++si)
        for (int64_t tg : targets) {
            if (shapes[si].steps == 2 && !two_step_ok(e)) continue;
            float ms = 0.f;
            int rc = time_choice(TuneChoice{shapes[si], tg}, 3, 3, &ms);
            if (rc) return rc;
            timed.emplace_back(ms, TuneChoice{shapes[si], tg});
        }
    // The leaders often lie within a percent or two of each other, where
    // one short timing can swap them: the three fastest are timed again,
    // round-robin (a drift of the clock then affects them alike), in longer
    // windows, and the lowest mean over the rounds wins (a run's speed is its
    // mean; the best single window favoured a march length that runs slower).
    std::stable_sort(timed.begin(), timed.end(),
                     [](const auto &x, const auto &y) { return x.first < y.first; });
    const size_t lead = std::min<size_t>(3, timed.size());
    std::vector<float> best_ms(lead, 0.f);
    for (int round = 0; round < 4; ++round)
        for (size_t c = 0; c < lead; ++c) {
            float ms = 0.f;
            int rc = time_choice(timed[c].second, 1, 12, &ms);
            if (rc) return rc;
            best_ms[c] += ms;
        }
    size_t win = 0;
    for (size_t c = 1; c < lead; ++c)
        if (best_ms[c] < best_ms[win]) win = c;
    if (lead > 0) choice = timed[win].second;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    e->tile = choice.tile;
    e->target_blocks = choice.target;
    drop_graphs(e);
    e->autotune = 1;
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        g_tune_cache[key] = choice;
    }
    return upload_desc(e);
}

int ens_run(fsc_ens *e, int64_t nsteps, int64_t sk_every) {
    TraceRange trace_("fsc run");
    if (nsteps < 0) return fail(e, FSC_E_INVAL, "nsteps < 0");
    if (nsteps == 0) return FSC_OK;
    if (e->step + nsteps > (int64_t(1) << 32)) return fail(e, FSC_E_INVAL, "step counter would pass 2^32");
    if (sk_every > 0) {
        for (auto &r : e->reps) {
            int rc = ensure_fft(r, e);
            if (rc) return rc;
        }
        int rc = ensure_measure_plan(e);
        if (rc) return rc;
    }
    if (e->autotune < 0) {
        int64_t nodes = 0;
        for (const auto &r : e->reps) nodes += r.N;
        if (e->autotune == -2 || nodes >= (int64_t(1) << 20)) {
            int rc = ens_autotune(e);
            if (rc) return rc;
        } else {
            e->autotune = 0;
        }
    }
    // whole chunks as graph replays; a graph holds the buffer of its first
    // launch, so a chunk must make an even number of launches (each launch
    // swaps the buffers)
    int64_t chunk = sk_every > 0 ? sk_every : 64;
    if (count_launches(e, chunk, sk_every) & 1) chunk *= 2;
    int64_t done = 0;
    const int64_t nchunks = nsteps / chunk;
    if (nchunks >= 2) {
        const int parity = e->cur;
        auto key = std::make_pair(parity, std::make_pair(chunk, sk_every));
        auto it = e->graphs.find(key);
        if (it == e->graphs.end()) {
            TraceRange trace_capture("fsc capture chunk");
            GraphEntry ge;
            hipGraph_t graph;
            HIPCHK(e, hipStreamBeginCapture(e->stream, hipStreamCaptureModeThreadLocal));
            int rc = enqueue_steps(e, parity, chunk, sk_every, &ge.samples, &ge.flips);
            hipError_t ec = hipStreamEndCapture(e->stream, &graph);
            if (rc) {
                if (ec == hipSuccess) (void)hipGraphDestroy(graph);
                return rc;
            }
            if (ge.flips) {
                (void)hipGraphDestroy(graph);
                return fail(e, FSC_E_STATE, "graph chunk with an odd number of launches");
            }
            if (ec != hipSuccess) return fail(e, FSC_E_HIP, std::string("capture: ") + hipGetErrorString(ec));
            ec = hipGraphInstantiate(&ge.exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (ec != hipSuccess) return fail(e, FSC_E_HIP, std::string("instantiate: ") + hipGetErrorString(ec));
            it = e->graphs.emplace(key, ge).first;
        }
        for (int64_t c = 0; c < nchunks; ++c) HIPCHK(e, hipGraphLaunch(it->second.exec, e->stream));
        for (auto &r : e->reps) r.nsamples += nchunks * it->second.samples;
        done = nchunks * chunk;
        e->step += done;
    }
    const int64_t rest = nsteps - done;
    if (rest > 0) {
        int64_t samples = 0;
        int flips = 0;
        int rc = enqueue_steps(e, e->cur, rest, sk_every, &samples, &flips);
        if (rc) return rc;
        e->cur ^= flips;
        for (auto &r : e->reps) r.nsamples += samples;
        e->step += rest;
    }
    return FSC_OK;
}

int ens_create(const fsc_params *ps, int nrep, void *stream, void *ext_a, void *ext_b,
               fsc_ens **out) {
    if (!out || !ps || nrep < 1) return FSC_E_INVAL;
    *out = nullptr;
    // validate everything before touching the device
    std::string err;
    std::vector<fsc_params> rp(nrep);
    for (int k = 0; k < nrep; ++k) {
        int rc = resolve_params(ps[k], rp[k], err);
        if (rc) {
            g_create_error = err;
            return rc;
        }
        if (rp[k].D != rp[0].D || rp[k].stencil != rp[0].stencil ||
            rp[k].precision != rp[0].precision) {
            g_create_error = "replicas must share D, stencil and precision";
            return FSC_E_INVAL;
        }
    }
    fsc_ens *e = new fsc_ens();
    e->stream = static_cast<hipStream_t>(stream);
    if (!e->stream) {
        // graphs cannot be captured on the null stream: use a private one
        if (hipStreamCreateWithFlags(&e->stream, hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            delete e;
            g_create_error = "stream creation failed";
            return FSC_E_HIP;
        }
        e->own_stream = true;
    }
    e->D = rp[0].D;
    e->stencil = rp[0].stencil;
    e->precision = rp[0].precision;
    TileShape shapes[32];
    tile_shapes(e->D, e->stencil, e->precision, shapes, 32);
    e->tile = shapes[0];
    if (const char *env = std::getenv("FSC_AUTOTUNE")) e->autotune = std::atoi(env) ? -2 : 0;
    e->reps.resize(nrep);
    for (int k = 0; k < nrep; ++k) {
        e->noise = e->noise || rp[k].kBT > 0.0;
        int rc = init_rep(e->reps[k], rp[k], ext_a, ext_b, e);
        if (rc) {
            g_create_error = e->err;
            ens_free(e);
            return rc;
        }
    }
    int rc = upload_desc(e);
    if (rc == FSC_OK) rc = set_step_device(e, 0);
    if (rc) {
        g_create_error = e->err;
        ens_free(e);
        return rc;
    }
    *out = e;
    return FSC_OK;
}

void ens_free(fsc_ens *e) {
    if (!e) return;
    (void)hipStreamSynchronize(e->stream);
    drop_graphs(e);
    for (auto &r : e->reps) {
        if (r.own) {
            if (r.buf[0]) (void)hipFree(r.buf[0]);
            if (r.buf[1]) (void)hipFree(r.buf[1]);
        }
        void *ptrs[] = {r.d_sk,     r.cbuf,       r.ctmp,  r.tw[0],     r.tw[1],      r.tw[2],
                        r.d_stats,  r.d_partials, r.d_mom, r.d_series, r.d_series_n, r.d_modes,
                        r.d_modes_n};
        for (void *p : ptrs)
            if (p) (void)hipFree(p);
    }
    if (e->d_desc) (void)hipFree(e->d_desc);
    if (e->d_tile_begin) (void)hipFree(e->d_tile_begin);
    if (e->d_step) (void)hipFree(e->d_step);
    if (e->d_meas) (void)hipFree(e->d_meas);
    if (e->d_mpre) (void)hipFree(e->d_mpre);
    if (e->own_stream) (void)hipStreamDestroy(e->stream);
    delete e;
}

int rep_index(fsc_ens *e, int replica) {
    if (replica < 0 || replica >= int(e->reps.size())) return fail(e, FSC_E_INVAL, "bad replica");
    return FSC_OK;
}

int ens_set_pop(fsc_ens *e, int ri, const double *host_f, int64_t step) {
    (void)step;
    Rep &r = e->reps[ri];
    const int nx = r.p.nx, ny = r.p.ny, nz = r.p.nz;
    const int par = e->cur;
    std::vector<unsigned char> raw(r.esz * size_t(r.Q) * size_t(r.N));
    for (int i = 0; i < r.Q; ++i) {
        const int cx = r.c[3 * i], cy = r.c[3 * i + 1], cz = r.c[3 * i + 2];
        const double shift = r.w[i] * r.p.rho0;
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    // stored f*_i(x) is the streamed f_i(x + c_i)
                    const int xs = wrap_any(x + cx, nx), ys = wrap_any(y + cy, ny), zs = wrap_any(z + cz, nz);
                    const size_t src = size_t(i) * r.N + xs + size_t(nx) * (ys + size_t(ny) * zs);
                    const size_t dst = size_t(i) * r.N + x + size_t(nx) * (y + size_t(ny) * z);
                    const double v = host_f[src] - shift;
                    if (r.esz == 4) reinterpret_cast<float *>(raw.data())[dst] = float(v);
                    else reinterpret_cast<double *>(raw.data())[dst] = v;
                }
    }
    HIPCHK(e, hipMemcpyAsync(r.buf[par], raw.data(), raw.size(), hipMemcpyHostToDevice, e->stream));
    HIPCHK(e, hipStreamSynchronize(e->stream));
    return FSC_OK;
}

int ens_get_pop(fsc_ens *e, int ri, double *host_f) {
    Rep &r = e->reps[ri];
    const int nx = r.p.nx, ny = r.p.ny, nz = r.p.nz;
    const int par = e->cur;
    std::vector<unsigned char> raw(r.esz * size_t(r.Q) * size_t(r.N));
    HIPCHK(e, hipMemcpyAsync(raw.data(), r.buf[par], raw.size(), hipMemcpyDeviceToHost, e->stream));
    HIPCHK(e, hipStreamSynchronize(e->stream));
    for (int i = 0; i < r.Q; ++i) {
        const int cx = r.c[3 * i], cy = r.c[3 * i + 1], cz = r.c[3 * i + 2];
        const double shift = r.w[i] * r.p.rho0;
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    const int xs = wrap_any(x - cx, nx), ys = wrap_any(y - cy, ny), zs = wrap_any(z - cz, nz);
                    const size_t src = size_t(i) * r.N + xs + size_t(nx) * (ys + size_t(ny) * zs);
                    const size_t dst = size_t(i) * r.N + x + size_t(nx) * (y + size_t(ny) * z);
                    const double v = r.esz == 4 ? double(reinterpret_cast<float *>(raw.data())[src])
                                                : reinterpret_cast<double *>(raw.data())[src];
                    host_f[dst] = shift + v;
                }
    }
    return FSC_OK;
}

int ens_stats(fsc_ens *e, int ri, double *out8) {
    Rep &r = e->reps[ri];
    HIPCHK(e, launch_stats(r.geom(), r.p.precision, r.buf[e->cur], r.p.rho0, r.d_partials,
                           r.d_stats, e->stream));
    HIPCHK(e, hipMemcpyAsync(out8, r.d_stats, sizeof(double) * 8, hipMemcpyDeviceToHost, e->stream));
    HIPCHK(e, hipStreamSynchronize(e->stream));
    if (out8[6] > 0.0) return fail(e, FSC_E_DIVERGED, "non-finite or non-positive density");
    return FSC_OK;
}

int ens_nbins(const fsc_ens *e, int ri, int kind, int *nbins) {
    const Rep &r = e->reps[ri];
    if (kind == FSC_SK_AXIS) *nbins = r.p.D * r.n_axis;
    else if (kind == FSC_SK_RADIAL) *nbins = r.n_rad;
    else return FSC_E_INVAL;
    return FSC_OK;
}

int ens_read_sk(fsc_ens *e, int ri, int kind, double *sum, double *sumsq, int64_t *count, int nbins) {
    Rep &r = e->reps[ri];
    int nb = 0;
    if (ens_nbins(e, ri, kind, &nb)) return fail(e, FSC_E_INVAL, "bad S(k) kind");
    if (nbins != nb) return fail(e, FSC_E_INVAL, "nbins does not match fsc_sk_nbins");
    if (nb == 0) return FSC_OK;
    const size_t na = size_t(r.p.D) * r.n_axis;
    const double *s = kind == FSC_SK_AXIS ? r.d_sk : r.d_sk + 2 * na;
    const double *q = kind == FSC_SK_AXIS ? r.d_sk + na : r.d_sk + 2 * na + r.n_rad;
    std::vector<double> hs(nb), hq(nb);
    StreamDrain drain{e->stream};
    HIPCHK(e, hipMemcpyAsync(hs.data(), s, sizeof(double) * nb, hipMemcpyDeviceToHost, e->stream));
    HIPCHK(e, hipMemcpyAsync(hq.data(), q, sizeof(double) * nb, hipMemcpyDeviceToHost, e->stream));
    HIPCHK(e, hipStreamSynchronize(e->stream));
    const auto &modes = kind == FSC_SK_AXIS ? r.axis_modes : r.rad_modes;
    for (int k = 0; k < nb; ++k) {
        if (sum) sum[k] = hs[k];
        if (sumsq) sumsq[k] = hq[k];
        if (count) count[k] = modes[k] * r.nsamples;
    }
    return FSC_OK;
}

int ens_sk_reset(fsc_ens *e) {
    for (auto &r : e->reps) {
        const size_t nsk = 2 * size_t(r.p.D) * r.n_axis + 2 * size_t(r.n_rad);
        HIPCHK(e, hipMemsetAsync(r.d_sk, 0, sizeof(double) * nsk, e->stream));
        r.nsamples = 0;
    }
    HIPCHK(e, hipStreamSynchronize(e->stream));
    return FSC_OK;
}

int ens_init_uniform(fsc_ens *e) {
    for (auto &r : e->reps) {
        const size_t bytes = r.esz * size_t(r.Q) * size_t(r.N);
        HIPCHK(e, hipMemsetAsync(r.buf[0], 0, bytes, e->stream));
        HIPCHK(e, hipMemsetAsync(r.buf[1], 0, bytes, e->stream));
    }
    e->cur = 0;
    int rc = set_step_device(e, 0);
    if (rc) return rc;
    return ens_sk_reset(e);
}

// Density n(x) of one replica's current state into host doubles [nz][ny][nx].
int ens_density(fsc_ens *e, int ri, double *host_rho) {
    Rep &r = e->reps[ri];
    void *tmp = nullptr;
    if (hipMalloc(&tmp, r.esz * size_t(r.N)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(e, FSC_E_OOM, "density buffer");
    }
    hipError_t ec = launch_density_real(r.geom(), r.p.precision, r.buf[e->cur], tmp, e->stream);
    std::vector<unsigned char> raw(r.esz * size_t(r.N));
    if (ec == hipSuccess) ec = hipMemcpyAsync(raw.data(), tmp, raw.size(), hipMemcpyDeviceToHost, e->stream);
    if (ec == hipSuccess) ec = hipStreamSynchronize(e->stream);
    (void)hipFree(tmp);
    if (ec != hipSuccess) return fail(e, FSC_E_HIP, hipGetErrorString(ec));
    for (int64_t s = 0; s < r.N; ++s)
        host_rho[s] = r.p.rho0 + (r.esz == 4 ? double(reinterpret_cast<float *>(raw.data())[s])
                                             : reinterpret_cast<double *>(raw.data())[s]);
    return FSC_OK;
}

// ---- checkpoints -----------------------------------------------------------
// File layout (native byte order): magic "FSCK", u32 version, u32 replica count,
// u32 zero, i64 step; then per replica: its resolved fsc_params, i64 S(k)
// sample count, u64 accumulator count, u64 population bytes, the populations
// exactly as stored (pull-layout deviations of the current buffer), the FP64
// S(k) accumulators.  Resuming from the file reproduces the run bit for bit,
// since the noise depends only on (seed, replica, node, step).
constexpr uint32_t kCkptMagic = 0x4b435346u;  // "FSCK" read as little-endian u32
constexpr uint32_t kCkptVersion = 1;

bool same_run(const fsc_params &a, const fsc_params &b) {
    auto eqd = [](double x, double y) { return std::memcmp(&x, &y, sizeof(double)) == 0; };
    return a.D == b.D && a.nx == b.nx && a.ny == b.ny && a.nz == b.nz && a.stencil == b.stencil &&
           a.precision == b.precision && eqd(a.G, b.G) && eqd(a.rho0, b.rho0) &&
           eqd(a.lambda_bulk, b.lambda_bulk) && eqd(a.lambda_shear, b.lambda_shear) &&
           eqd(a.lambda_ghost, b.lambda_ghost) && eqd(a.kBT, b.kBT) && a.seed == b.seed &&
           a.replica == b.replica;
}

uint64_t sk_len(const Rep &r) { return 2 * uint64_t(r.p.D) * r.n_axis + 2 * uint64_t(r.n_rad); }

int ens_save(fsc_ens *e, const char *path) {
    std::unique_ptr<FILE, int (*)(FILE *)> fp(std::fopen(path, "wb"), std::fclose);
    if (!fp) return fail(e, FSC_E_IO, std::string("cannot open ") + path + " for writing");
    auto put = [&](const void *p, size_t n) { return std::fwrite(p, 1, n, fp.get()) == n; };
    const uint32_t head[4] = {kCkptMagic, kCkptVersion, uint32_t(e->reps.size()), 0};
    bool ok = put(head, sizeof(head)) && put(&e->step, sizeof(e->step));
    const int par = e->cur;
    std::vector<unsigned char> raw;
    std::vector<double> acc;
    StreamDrain drain{e->stream};
    for (size_t k = 0; ok && k < e->reps.size(); ++k) {
        Rep &r = e->reps[k];
        const uint64_t nsk = sk_len(r);
        const uint64_t nbytes = uint64_t(r.esz) * r.Q * r.N;
        raw.resize(nbytes);
        acc.resize(nsk);
        HIPCHK(e, hipMemcpyAsync(raw.data(), r.buf[par], nbytes, hipMemcpyDeviceToHost, e->stream));
        HIPCHK(e, hipMemcpyAsync(acc.data(), r.d_sk, sizeof(double) * nsk, hipMemcpyDeviceToHost,
                                 e->stream));
        HIPCHK(e, hipStreamSynchronize(e->stream));
        ok = put(&r.p, sizeof(r.p)) && put(&r.nsamples, sizeof(r.nsamples)) && put(&nsk, sizeof(nsk)) &&
             put(&nbytes, sizeof(nbytes)) && put(raw.data(), nbytes) &&
             put(acc.data(), sizeof(double) * nsk);
    }
    if (!ok || std::fflush(fp.get()) != 0) return fail(e, FSC_E_IO, std::string("write failed: ") + path);
    return FSC_OK;
}

int ens_load(fsc_ens *e, const char *path) {
    std::unique_ptr<FILE, int (*)(FILE *)> fp(std::fopen(path, "rb"), std::fclose);
    if (!fp) return fail(e, FSC_E_IO, std::string("cannot open ") + path);
    auto get = [&](void *p, size_t n) { return std::fread(p, 1, n, fp.get()) == n; };
    uint32_t head[4];
    int64_t step = 0;
    if (!get(head, sizeof(head)) || !get(&step, sizeof(step)) || head[0] != kCkptMagic)
        return fail(e, FSC_E_IO, std::string("not a checkpoint: ") + path);
    if (head[1] != kCkptVersion) return fail(e, FSC_E_IO, "unsupported checkpoint version");
    if (head[2] != e->reps.size()) return fail(e, FSC_E_INVAL, "checkpoint holds another replica count");
    if (step < 0) return fail(e, FSC_E_IO, "corrupt checkpoint step");
    // read and check the whole file before any device state changes
    const size_t n = e->reps.size();
    std::vector<std::vector<unsigned char>> raws(n);
    std::vector<std::vector<double>> accs(n);
    std::vector<int64_t> ns(n);
    for (size_t k = 0; k < n; ++k) {
        const Rep &r = e->reps[k];
        fsc_params p;
        uint64_t nsk = 0, nbytes = 0;
        if (!get(&p, sizeof(p)) || !get(&ns[k], sizeof(int64_t)) || !get(&nsk, sizeof(nsk)) ||
            !get(&nbytes, sizeof(nbytes)))
            return fail(e, FSC_E_IO, "truncated checkpoint");
        if (!same_run(p, r.p))
            return fail(e, FSC_E_INVAL,
                        "checkpoint replica " + std::to_string(k) + " was written with other parameters");
        if (nsk != sk_len(r) || nbytes != uint64_t(r.esz) * r.Q * r.N || ns[k] < 0)
            return fail(e, FSC_E_IO, "checkpoint sizes do not match the lattice");
        raws[k].resize(nbytes);
        accs[k].resize(nsk);
        if (!get(raws[k].data(), nbytes) || !get(accs[k].data(), sizeof(double) * nsk))
            return fail(e, FSC_E_IO, "truncated checkpoint");
    }
    // the host vectors must outlive the copies: wait for the stream before
    // returning, also after a failed call
    const int par = e->cur;
    hipError_t ec = hipSuccess;
    for (size_t k = 0; k < n && ec == hipSuccess; ++k) {
        Rep &r = e->reps[k];
        ec = hipMemcpyAsync(r.buf[par], raws[k].data(), raws[k].size(), hipMemcpyHostToDevice, e->stream);
        if (ec == hipSuccess)
            ec = hipMemcpyAsync(r.d_sk, accs[k].data(), sizeof(double) * accs[k].size(),
                                hipMemcpyHostToDevice, e->stream);
    }
    const hipError_t es = hipStreamSynchronize(e->stream);
    if (ec == hipSuccess) ec = es;
    if (ec != hipSuccess) return fail(e, FSC_E_HIP, std::string("checkpoint upload: ") + hipGetErrorString(ec));
    for (size_t k = 0; k < n; ++k) e->reps[k].nsamples = ns[k];
    return set_step_device(e, step);
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char *fsc_strerror(int code) {
    switch (code) {
    case FSC_OK: return "ok";
    case FSC_E_INVAL: return "invalid argument";
    case FSC_E_HIP: return "HIP runtime error";
    case FSC_E_OOM: return "out of memory";
    case FSC_E_DIVERGED: return "diverged (non-finite or non-positive density)";
    case FSC_E_STATE: return "invalid state";
    case FSC_E_NOTSUP: return "not supported";
    case FSC_E_IO: return "file error";
    case FSC_E_RANGE: return "input larger than the fixed-size scratch allows";
    default: return "unknown error";
    }
}

int fsc_create(const fsc_params *p, void *stream, fsc_ctx **out) {
    return fsc_create_external(p, stream, nullptr, nullptr, out);
}

int fsc_create_external(const fsc_params *p, void *stream, void *a, void *b, fsc_ctx **out) {
    if (!out || !p) return FSC_E_INVAL;
    *out = nullptr;
    fsc_ens *e = nullptr;
    int rc = ens_create(p, 1, stream, a, b, &e);
    if (rc) return rc;
    *out = new fsc_ctx{e};
    return FSC_OK;
}

int fsc_destroy(fsc_ctx *ctx) {
    if (!ctx) return FSC_E_INVAL;
    ens_free(ctx->e);
    delete ctx;
    return FSC_OK;
}

const char *fsc_last_error(const fsc_ctx *ctx) {
    return ctx ? ctx->e->err.c_str() : g_create_error.c_str();
}

int fsc_get_params(const fsc_ctx *ctx, fsc_params *out) {
    if (!ctx || !out) return FSC_E_INVAL;
    *out = ctx->e->reps[0].p;
    return FSC_OK;
}

int fsc_init_uniform(fsc_ctx *ctx) {
    if (!ctx) return FSC_E_INVAL;
    return ens_init_uniform(ctx->e);
}

int fsc_set_populations(fsc_ctx *ctx, const double *host_f, int64_t step) {
    if (!ctx || !host_f) return FSC_E_INVAL;
    if (step < 0 || step >= (int64_t(1) << 32)) return fail(ctx->e, FSC_E_INVAL, "step out of range");
    int rc = ens_set_pop(ctx->e, 0, host_f, step);
    if (rc) return rc;
    return set_step_device(ctx->e, step);
}

int fsc_get_populations(fsc_ctx *ctx, double *host_f, int64_t *step) {
    if (!ctx || !host_f) return FSC_E_INVAL;
    if (step) *step = ctx->e->step;
    return ens_get_pop(ctx->e, 0, host_f);
}

int fsc_step(fsc_ctx *ctx, int64_t nsteps) {
    if (!ctx) return FSC_E_INVAL;
    return ens_run(ctx->e, nsteps, 0);
}

int fsc_run(fsc_ctx *ctx, int64_t nsteps, int64_t sk_every) {
    if (!ctx) return FSC_E_INVAL;
    return ens_run(ctx->e, nsteps, sk_every);
}

int fsc_get_step(const fsc_ctx *ctx, int64_t *step) {
    if (!ctx || !step) return FSC_E_INVAL;
    *step = ctx->e->step;
    return FSC_OK;
}

int fsc_density(fsc_ctx *ctx, double *host_rho) {
    if (!ctx || !host_rho) return FSC_E_INVAL;
    return ens_density(ctx->e, 0, host_rho);
}

int fsc_read_density(fsc_ctx *ctx, double *host_rho) { return fsc_density(ctx, host_rho); }

int fsc_stats(fsc_ctx *ctx, double *out8) {
    if (!ctx || !out8) return FSC_E_INVAL;
    return ens_stats(ctx->e, 0, out8);
}

int fsc_conserved(fsc_ctx *ctx, double *mass, double *mom) {
    if (!ctx || !mass || !mom) return FSC_E_INVAL;
    double out[8];
    const int rc = ens_stats(ctx->e, 0, out);
    if (rc != FSC_OK && rc != FSC_E_DIVERGED) return rc;
    *mass = out[0];
    for (int d = 0; d < ctx->e->reps[0].p.D; ++d) mom[d] = out[1 + d];
    return rc;
}

int fsc_sk_reset(fsc_ctx *ctx) {
    if (!ctx) return FSC_E_INVAL;
    return ens_sk_reset(ctx->e);
}

int fsc_measure_sk(fsc_ctx *ctx) {
    TraceRange trace_("fsc measure_sk");
    if (!ctx) return FSC_E_INVAL;
    fsc_ens *e = ctx->e;
    Rep &r = e->reps[0];
    int rc = ensure_fft(r, e);
    if (rc) return rc;
    rc = ensure_measure_plan(e);
    if (rc) return rc;
    rc = enqueue_measure(e, e->cur, 0);
    if (rc) return rc;
    r.nsamples += 1;
    return FSC_OK;
}

int fsc_sk_nbins(const fsc_ctx *ctx, int kind, int *nbins) {
    if (!ctx || !nbins) return FSC_E_INVAL;
    return ens_nbins(ctx->e, 0, kind, nbins);
}

int fsc_read_sk(fsc_ctx *ctx, int kind, double *sum, double *sumsq, int64_t *count, int nbins) {
    if (!ctx) return FSC_E_INVAL;
    return ens_read_sk(ctx->e, 0, kind, sum, sumsq, count, nbins);
}

// ---- ensemble -------------------------------------------------------------
int fsc_ens_create(const fsc_params *reps, int nrep, void *stream, fsc_ens **out) {
    return ens_create(reps, nrep, stream, nullptr, nullptr, out);
}
int fsc_ens_destroy(fsc_ens *ens) {
    if (!ens) return FSC_E_INVAL;
    ens_free(ens);
    return FSC_OK;
}
const char *fsc_ens_last_error(const fsc_ens *ens) {
    return ens ? ens->err.c_str() : g_create_error.c_str();
}
int fsc_ens_init_uniform(fsc_ens *ens) { return ens ? ens_init_uniform(ens) : FSC_E_INVAL; }
int fsc_ens_run(fsc_ens *ens, int64_t nsteps, int64_t sk_every) {
    return ens ? ens_run(ens, nsteps, sk_every) : FSC_E_INVAL;
}
int fsc_ens_get_step(const fsc_ens *ens, int64_t *step) {
    if (!ens || !step) return FSC_E_INVAL;
    *step = ens->step;
    return FSC_OK;
}
int fsc_ens_get_populations(fsc_ens *ens, int replica, double *host_f) {
    if (!ens || !host_f) return FSC_E_INVAL;
    int rc = rep_index(ens, replica);
    return rc ? rc : ens_get_pop(ens, replica, host_f);
}
int fsc_ens_set_populations(fsc_ens *ens, int replica, const double *host_f) {
    if (!ens || !host_f) return FSC_E_INVAL;
    int rc = rep_index(ens, replica);
    return rc ? rc : ens_set_pop(ens, replica, host_f, ens->step);
}
int fsc_ens_stats(fsc_ens *ens, int replica, double *out8) {
    if (!ens || !out8) return FSC_E_INVAL;
    int rc = rep_index(ens, replica);
    return rc ? rc : ens_stats(ens, replica, out8);
}
int fsc_ens_sk_nbins(const fsc_ens *ens, int replica, int kind, int *nbins) {
    if (!ens || !nbins || replica < 0 || replica >= int(ens->reps.size())) return FSC_E_INVAL;
    return ens_nbins(ens, replica, kind, nbins);
}
int fsc_ens_read_sk(fsc_ens *ens, int replica, int kind, double *sum, double *sumsq, int64_t *count,
                    int nbins) {
    if (!ens) return FSC_E_INVAL;
    int rc = rep_index(ens, replica);
    return rc ? rc : ens_read_sk(ens, replica, kind, sum, sumsq, count, nbins);
}
int fsc_ens_sk_reset(fsc_ens *ens) { return ens ? ens_sk_reset(ens) : FSC_E_INVAL; }
int fsc_ens_density(fsc_ens *ens, int replica, double *host_rho) {
    if (!ens || !host_rho) return FSC_E_INVAL;
    int rc = rep_index(ens, replica);
    return rc ? rc : ens_density(ens, replica, host_rho);
}
int fsc_ens_save(fsc_ens *ens, const char *path) {
    return ens && path ? ens_save(ens, path) : FSC_E_INVAL;
}
int fsc_ens_load(fsc_ens *ens, const char *path) {
    return ens && path ? ens_load(ens, path) : FSC_E_INVAL;
}
int fsc_save(fsc_ctx *ctx, const char *path) {
    return ctx && path ? ens_save(ctx->e, path) : FSC_E_INVAL;
}
int fsc_load(fsc_ctx *ctx, const char *path) {
    return ctx && path ? ens_load(ctx->e, path) : FSC_E_INVAL;
}

// ---- time series ----------------------------------------------------------
int fsc_series_enable(fsc_ctx *ctx, int capacity) {
    if (!ctx || capacity < 0) return FSC_E_INVAL;
    drop_graphs(ctx->e);
    return series_enable(ctx->e, ctx->e->reps[0], capacity);
}
int fsc_read_series(fsc_ctx *ctx, double *out, int max_rows, int *nrows, int *row_len) {
    if (!ctx) return FSC_E_INVAL;
    return series_read(ctx->e, ctx->e->reps[0], out, max_rows, nrows, row_len);
}
int fsc_ens_series_enable(fsc_ens *ens, int capacity) {
    if (!ens || capacity < 0) return FSC_E_INVAL;
    drop_graphs(ens);
    for (auto &r : ens->reps) {
        int rc = series_enable(ens, r, capacity);
        if (rc) return rc;
    }
    return FSC_OK;
}
int fsc_ens_read_series(fsc_ens *ens, int replica, double *out, int max_rows, int *nrows,
                        int *row_len) {
    if (!ens) return FSC_E_INVAL;
    int rc = rep_index(ens, replica);
    return rc ? rc : series_read(ens, ens->reps[replica], out, max_rows, nrows, row_len);
}

// ---- recorded mode amplitudes ---------------------------------------------------
int fsc_modes_enable(fsc_ctx *ctx, int nm, int capacity) {
    if (!ctx || capacity < 0 || (capacity > 0 && nm < 1)) return FSC_E_INVAL;
    drop_graphs(ctx->e);
    return modes_enable(ctx->e, ctx->e->reps[0], nm, capacity);
}
int fsc_read_modes(fsc_ctx *ctx, double *out, int max_rows, int *nrows) {
    if (!ctx) return FSC_E_INVAL;
    return modes_read(ctx->e, ctx->e->reps[0], out, max_rows, nrows);
}
int fsc_ens_modes_enable(fsc_ens *ens, int nm, int capacity) {
    if (!ens || capacity < 0 || (capacity > 0 && nm < 1)) return FSC_E_INVAL;
    drop_graphs(ens);
    for (auto &r : ens->reps) {
        int rc = modes_enable(ens, r, nm, capacity);
        if (rc) return rc;
    }
    return FSC_OK;
}
int fsc_ens_read_modes(fsc_ens *ens, int replica, double *out, int max_rows, int *nrows) {
    if (!ens) return FSC_E_INVAL;
    int rc = rep_index(ens, replica);
    return rc ? rc : modes_read(ens, ens->reps[replica], out, max_rows, nrows);
}

// ---- tiling ---------------------------------------------------------------
int fsc_autotune(fsc_ctx *ctx) { return ctx ? ens_autotune(ctx->e) : FSC_E_INVAL; }
int fsc_ens_autotune(fsc_ens *ens) { return ens ? ens_autotune(ens) : FSC_E_INVAL; }
static int get_tiling(const fsc_ens *e, int *out5) {
    if (!out5) return FSC_E_INVAL;
    out5[0] = e->tile.tx;
    out5[1] = e->tile.ty;
    out5[2] = e->tile.pf;
    out5[3] = e->total_tiles;
    out5[4] = e->tile.steps;
    return FSC_OK;
}
int fsc_get_tiling(const fsc_ctx *ctx, int *out5) { return ctx ? get_tiling(ctx->e, out5) : FSC_E_INVAL; }
int fsc_ens_get_tiling(const fsc_ens *ens, int *out5) { return ens ? get_tiling(ens, out5) : FSC_E_INVAL; }

int fsc_tile_shapes(int D, int stencil, int precision, int *out4, int max) {
    if (!((D == 2 && (stencil == FSC_E4 || stencil == FSC_E8)) || (D == 3 && stencil == FSC_E4)) ||
        (precision != FSC_FP32_SHIFTED && precision != FSC_FP64) || max < 0 || (max > 0 && !out4))
        return FSC_E_INVAL;
    TileShape t[32];
    const int n = tile_shapes(D, stencil, precision, t, 32);
    for (int i = 0; i < n && i < max; ++i) {
        out4[4 * i] = t[i].tx;
        out4[4 * i + 1] = t[i].ty;
        out4[4 * i + 2] = t[i].pf;
        out4[4 * i + 3] = t[i].steps;
    }
    return n;
}

static int set_tiling(fsc_ens *e, int tx, int ty, int pf, int steps, int64_t target_blocks) {
    if (target_blocks < 1) return fail(e, FSC_E_INVAL, "target_blocks < 1");
    TileShape t[32];
    const int n = tile_shapes(e->D, e->stencil, e->precision, t, 32);
    for (int i = 0; i < n; ++i)
        if (t[i].tx == tx && t[i].ty == ty && t[i].pf == pf && t[i].steps == steps) {
            if (steps == 2 && !two_step_ok(e))
                return fail(e, FSC_E_INVAL,
                            "two-step tiling needs sides of at least 2R + 2 columns and buffers below 4 GiB");
            e->tile = t[i];
            e->target_blocks = target_blocks;
            drop_graphs(e);
            e->autotune = 1;  // an explicit choice is never re-tuned
            return upload_desc(e);
        }
    return fail(e, FSC_E_INVAL, "tile shape not compiled for this lattice (see fsc_tile_shapes)");
}
int fsc_set_tiling(fsc_ctx *ctx, int tx, int ty, int pf, int steps, int64_t target_blocks) {
    return ctx ? set_tiling(ctx->e, tx, ty, pf, steps, target_blocks) : FSC_E_INVAL;
}
int fsc_ens_set_tiling(fsc_ens *ens, int tx, int ty, int pf, int steps, int64_t target_blocks) {
    return ens ? set_tiling(ens, tx, ty, pf, steps, target_blocks) : FSC_E_INVAL;
}

// ---- coarse-graining and field measurement (surrogate inputs/outputs) ---
int fsc_coarsen(fsc_ctx *ctx, int factor, float *dev_out) {
    if (!ctx || !dev_out) return FSC_E_INVAL;
    fsc_ens *e = ctx->e;
    Rep &r = e->reps[0];
    if (r.p.D != 2 || factor < 1 || r.p.nx % factor || r.p.ny % factor)
        return fail(e, FSC_E_INVAL, "coarsening needs a 2D lattice with sides divisible by factor");
    HIPCHK(e, launch_coarsen(r.geom(), r.p.precision, r.buf[e->cur], r.p.rho0, factor, dev_out,
                             e->stream));
    return FSC_OK;
}

int fsc_ens_coarsen(fsc_ens *ens, int replica, int factor, float *dev_out) {
    if (!ens || !dev_out) return FSC_E_INVAL;
    int rc = rep_index(ens, replica);
    if (rc) return rc;
    Rep &r = ens->reps[replica];
    if (r.p.D != 2 || factor < 1 || r.p.nx % factor || r.p.ny % factor)
        return fail(ens, FSC_E_INVAL, "coarsening needs a 2D lattice with sides divisible by factor");
    HIPCHK(ens, launch_coarsen(r.geom(), r.p.precision, r.buf[ens->cur], r.p.rho0, factor,
                               dev_out, ens->stream));
    return FSC_OK;
}

namespace {

// Shell index round(sqrt(m)) of a squared mode number, in integer arithmetic.
int round_sqrt_shell(int64_t m) {
    int64_t b = int64_t(std::sqrt(double(m)));
    while (b * b > m) --b;
    while ((b + 1) * (b + 1) <= m) ++b;
    if (m - b * b > b) ++b;
    return int(b);
}

// Mode count of each radial shell of an L x L box (k = 0 excluded).
void field_shell_modes(int L, int nrad, int64_t *modes) {
    for (int k = 0; k < nrad; ++k) modes[k] = 0;
    for (int y = 0; y < L; ++y)
        for (int x = 0; x < L; ++x) {
            const int64_t mx = x <= L / 2 ? x : x - L, my = y <= L / 2 ? y : y - L;
            if (mx || my) modes[round_sqrt_shell(mx * mx + my * my)] += 1;
        }
}

// Device work areas of one field S(k): two complex lines of N points, the
// twiddles, the FP64 bin accumulators and the series counter.
struct FieldWork {
    void *ca, *cb, *tw;
    double *acc;
    int *cnt;
};

size_t field_acc_len(int L, int nrad) {
    return 2 * size_t(2 * (L / 2 + 1)) + 2 * size_t(nrad) + 2 + size_t(2 + nrad);
}

// S(k) of `batch` fields [batch][L][L] (float) on stream st, one field after
// the other through the work areas w: density to complex, FFT along x then
// y, radial binning with the first moment, then the shell sums and the moment
// pair are copied to the host.  Shared by fsc_field_sk (which allocates w per
// call) and fsc_field_sk_noalloc (which uses the library's static scratch).
hipError_t field_sk_batches(const float *dev_fields, int batch, int L, hipStream_t st,
                            const FieldWork &w, const int64_t *modes, int nrad,
                            double *host_shell_mean, double *host_L) {
    const int64_t N = int64_t(L) * L;
    const int na = L / 2 + 1;
    const size_t nacc = field_acc_len(L, nrad);
    hipError_t ec = launch_twiddles(0, w.tw, L, st);
    const Geometry g{2, L, L, 1, N};
    for (int b = 0; b < batch && ec == hipSuccess; ++b) {
        // the accumulators and the series counter start at zero for every field
        ec = launch_zero_words(w.acc, int64_t(2 * nacc), st);
        if (ec == hipSuccess) ec = launch_zero_words(w.cnt, 1, st);
        if (ec == hipSuccess) ec = launch_field_cplx(dev_fields + size_t(b) * N, int(N), w.ca, st);
        if (ec == hipSuccess) ec = launch_fft_axis(0, w.ca, w.cb, w.tw, L, L, 1, st);
        if (ec == hipSuccess) ec = launch_fft_axis(0, w.cb, w.ca, w.tw, L, L, 1, st);
        BinTargets t;
        t.axis_sum = w.acc;
        t.axis_sq = w.acc + 2 * na;
        t.rad_sum = w.acc + 4 * na;
        t.rad_sq = w.acc + 4 * na + nrad;
        t.n_axis = na;
        t.n_rad = nrad;
        t.mom = w.acc + 4 * na + 2 * nrad;
        t.series = w.acc + 4 * na + 2 * nrad + 2;
        t.series_n = w.cnt;
        t.series_cap = 1;
        if (ec == hipSuccess) ec = launch_bin(g, 0, w.ca, t, st);
        double mom[2] = {0.0, 0.0};
        double *shell = host_shell_mean ? host_shell_mean + size_t(b) * nrad : nullptr;
        if (ec == hipSuccess && shell)
            ec = hipMemcpyAsync(shell, t.rad_sum, sizeof(double) * nrad, hipMemcpyDeviceToHost, st);
        if (ec == hipSuccess)
            ec = hipMemcpyAsync(mom, t.mom, sizeof(mom), hipMemcpyDeviceToHost, st);
        if (ec == hipSuccess) ec = hipStreamSynchronize(st);
        if (ec != hipSuccess) break;
        if (shell)
            for (int k = 0; k < nrad; ++k) shell[k] = modes[k] ? shell[k] / double(modes[k]) : 0.0;
        if (host_L) host_L[b] = mom[1] > 0.0 ? 2.0 * M_PI * mom[0] / mom[1] : 0.0;
    }
    return ec;
}

// ---- fixed-size scratch of the allocation-free field S(k) ----------------
// Sized for fields up to FIELD_STATIC_MAX_SIDE^2: two complex work lines of
// 8 B per point, the twiddles, the accumulators and the counter, each at a
// 256-byte boundary.  Every device the library runs on holds one copy for the
// life of the process.
constexpr int FIELD_STATIC_MAX_SIDE = 1024;
constexpr int FIELD_STATIC_MAX_NRAD = 726;  // round(sqrt(2) * 512) + 1
constexpr size_t align256(size_t v) { return (v + 255) & ~size_t(255); }
constexpr size_t FS_CPLX = 8 * size_t(FIELD_STATIC_MAX_SIDE) * FIELD_STATIC_MAX_SIDE;
constexpr size_t FS_TW = align256(8 * size_t(FIELD_STATIC_MAX_SIDE));
constexpr size_t FS_ACC = align256(8 * (2 * size_t(2 * (FIELD_STATIC_MAX_SIDE / 2 + 1)) +
                                        2 * size_t(FIELD_STATIC_MAX_NRAD) + 2 +
                                        size_t(2 + FIELD_STATIC_MAX_NRAD)));
constexpr size_t FS_BYTES = 2 * FS_CPLX + FS_TW + FS_ACC + 256;

__device__ __align__(256) unsigned char scratch[FS_BYTES];

constexpr int FS_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[FS_MAX_DEVICES] = {};

// Device address of `scratch` on device dev, looked up once per device with
// that device current (the array's host-side name is not a device address).
hipError_t scratch_on(int dev, void **out) {
    if (dev < 0 || dev >= FS_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        int prev = -1;
        hipError_t ec = hipGetDevice(&prev);
        if (ec != hipSuccess) return ec;
        if (prev != dev && (ec = hipSetDevice(dev)) != hipSuccess) return ec;
        void *ptr = nullptr;
        ec = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (prev != dev) (void)hipSetDevice(prev);
        if (ec != hipSuccess) return ec;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

int field_args(const float *dev_fields, int batch, int ny, int nx, int nbins, int *nrad) {
    if (!dev_fields || batch < 1 || nx < 2 || ny < 2 || nx != ny || nx > 8192) return FSC_E_INVAL;
    *nrad = round_sqrt_shell(2 * int64_t(nx / 2) * (nx / 2)) + 1;
    return nbins == *nrad ? FSC_OK : FSC_E_INVAL;
}

}  // namespace

int fsc_field_sk(const float *dev_fields, int batch, int ny, int nx, void *stream,
                 double *host_shell_mean, double *host_L, int nbins) {
    int nrad = 0;
    int rc = field_args(dev_fields, batch, ny, nx, nbins, &nrad);
    if (rc) return rc;
    const hipStream_t st = static_cast<hipStream_t>(stream);
    const int L = nx;
    std::vector<int64_t> modes(nrad, 0);
    field_shell_modes(L, nrad, modes.data());
    const int64_t N = int64_t(L) * L;
    void *ca = nullptr, *cb = nullptr, *tw = nullptr;
    double *acc = nullptr;
    int *cnt = nullptr;
    const size_t nacc = field_acc_len(L, nrad);
    if (hipMalloc(&ca, 8 * N) != hipSuccess || hipMalloc(&cb, 8 * N) != hipSuccess ||
        hipMalloc(&tw, 8 * twiddle_len(L)) != hipSuccess ||
        hipMalloc(&acc, sizeof(double) * nacc) != hipSuccess ||
        hipMalloc(&cnt, sizeof(int)) != hipSuccess) {
        (void)hipGetLastError();
        for (void *p : {ca, cb, tw, (void *)acc, (void *)cnt})
            if (p) (void)hipFree(p);
        return FSC_E_OOM;
    }
    const FieldWork w{ca, cb, tw, acc, cnt};
    hipError_t ec = field_sk_batches(dev_fields, batch, L, st, w, modes.data(), nrad,
                                     host_shell_mean, host_L);
    for (void *p : {ca, cb, tw, (void *)acc, (void *)cnt}) (void)hipFree(p);
    return ec == hipSuccess ? FSC_OK : FSC_E_HIP;
}

int fsc_field_sk_noalloc(const float *dev_fields, int batch, int ny, int nx, void *stream,
                         double *host_shell_mean, double *host_L, int nbins) {
    int nrad = 0;
    int rc = field_args(dev_fields, batch, ny, nx, nbins, &nrad);
    if (rc) return rc;
    if (nx > FIELD_STATIC_MAX_SIDE) return FSC_E_RANGE;
    const hipStream_t st = static_cast<hipStream_t>(stream);
    int dev = -1;
    hipError_t ec = st ? hipStreamGetDevice(st, &dev) : hipGetDevice(&dev);
    if (ec != hipSuccess) return FSC_E_HIP;
    void *base = nullptr;
    if (scratch_on(dev, &base) != hipSuccess) return FSC_E_HIP;
    unsigned char *p = static_cast<unsigned char *>(base);
    const FieldWork w{p, p + FS_CPLX, p + 2 * FS_CPLX,
                      reinterpret_cast<double *>(p + 2 * FS_CPLX + FS_TW),
                      reinterpret_cast<int *>(p + 2 * FS_CPLX + FS_TW + FS_ACC)};
    int64_t modes[FIELD_STATIC_MAX_NRAD];
    field_shell_modes(nx, nrad, modes);
    ec = field_sk_batches(dev_fields, batch, nx, st, w, modes, nrad, host_shell_mean, host_L);
    return ec == hipSuccess ? FSC_OK : FSC_E_HIP;
}

int fsc_field_nbins(int n, int *nbins) {
    if (n < 2 || !nbins) return FSC_E_INVAL;
    int64_t m = 2 * int64_t(n / 2) * (n / 2);
    int64_t b = int64_t(std::sqrt(double(m)));
    while (b * b > m) --b;
    while ((b + 1) * (b + 1) <= m) ++b;
    if (m - b * b > b) ++b;
    *nbins = int(b) + 1;
    return FSC_OK;
}

// ---- diagnostics ----------------------------------------------------------
int fsc_copy(const void *dev_src, void *dev_dst, int64_t bytes, void *stream) {
    if (!dev_src || !dev_dst || bytes <= 0 || (bytes & 15)) return FSC_E_INVAL;
    return launch_copy(dev_src, dev_dst, bytes, static_cast<hipStream_t>(stream)) == hipSuccess
               ? FSC_OK
               : FSC_E_HIP;
}

// ---- generator checks ---------------------------------------------------
int fsc_philox(const uint32_t *host_ctr, const uint32_t *host_key, uint32_t *host_out, int64_t n) {
    if (n < 0 || (n > 0 && (!host_ctr || !host_key || !host_out))) return FSC_E_INVAL;
    if (n == 0) return FSC_OK;
    uint32_t *d = nullptr;
    const size_t bytes = sizeof(uint32_t) * size_t(n) * 10;
    if (hipMalloc(&d, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return FSC_E_OOM;
    }
    hipError_t ec = hipMemcpy(d, host_ctr, sizeof(uint32_t) * 4 * n, hipMemcpyHostToDevice);
    if (ec == hipSuccess) ec = hipMemcpy(d + 4 * n, host_key, sizeof(uint32_t) * 2 * n, hipMemcpyHostToDevice);
    if (ec == hipSuccess) ec = launch_philox(d, d + 4 * n, d + 6 * n, n, nullptr);
    if (ec == hipSuccess) ec = hipMemcpy(host_out, d + 6 * n, sizeof(uint32_t) * 4 * n, hipMemcpyDeviceToHost);
    (void)hipFree(d);
    return ec == hipSuccess ? FSC_OK : FSC_E_HIP;
}

int fsc_normals(int D, int precision, uint64_t seed, uint32_t replica, const int64_t *host_node,
                const int64_t *host_step, int64_t n, double *host_out) {
    if ((D != 2 && D != 3) || (precision != 0 && precision != 1) || n < 0) return FSC_E_INVAL;
    if (n == 0) return FSC_OK;
    if (!host_node || !host_step || !host_out) return FSC_E_INVAL;
    const int nn = D == 2 ? D2Q9::NNORM : D3Q19::NNORM;
    int64_t *d = nullptr;
    const size_t bytes = sizeof(int64_t) * size_t(n) * 2 + sizeof(double) * size_t(n) * nn;
    if (hipMalloc(&d, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return FSC_E_OOM;
    }
    double *dout = reinterpret_cast<double *>(d + 2 * n);
    hipError_t ec = hipMemcpy(d, host_node, sizeof(int64_t) * n, hipMemcpyHostToDevice);
    if (ec == hipSuccess) ec = hipMemcpy(d + n, host_step, sizeof(int64_t) * n, hipMemcpyHostToDevice);
    if (ec == hipSuccess) ec = launch_normals(D, precision, seed, replica, d, d + n, n, dout, nullptr);
    if (ec == hipSuccess) ec = hipMemcpy(host_out, dout, sizeof(double) * n * nn, hipMemcpyDeviceToHost);
    (void)hipFree(d);
    return ec == hipSuccess ? FSC_OK : FSC_E_HIP;
}

}  // extern "C"

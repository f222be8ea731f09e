// Stage sequencing of the synthesis Y = N F D S (Eq. 5) and the adjoint Y^H = S^H D^H F^H N^H
// (Eq. 6) of arXiv:2406.14542 on one HIP stream, with rocFFT for the uniform FFTs.
// Everything is enqueued asynchronously; intermediates live in two ping-pong scratch
// regions X and Y (and Z for the spreading subgrids) that the plan owns.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "internal.h"

namespace nusht {

int interp_f64(const nusht_plan_s* p, const double* fine, double* out, int nmaps, hipStream_t s);
int interp_f32(const nusht_plan_s* p, const float* fine, double* out, int nmaps, hipStream_t s);
int spread_group_f64(const nusht_plan_s* p, const double* vals, double* fine, int mb,
                     hipStream_t s);
int spread_group_f32(const nusht_plan_s* p, const double* vals, float* fine, int mb,
                     hipStream_t s);

namespace {

std::once_flag g_fft_once;

int make_fft(FftPlan& f, rocfft_transform_type type, rocfft_precision prec, size_t dim,
             const size_t* lengths, size_t batch, rocfft_result_placement place)
{
    rocfft_plan_description desc = nullptr;
    NUSHT_FFT(rocfft_plan_description_create(&desc));
    if (type == rocfft_transform_type_real_forward || type == rocfft_transform_type_real_inverse) {
        // default packed layouts for real transforms
        rocfft_array_type in_t = type == rocfft_transform_type_real_forward
                                     ? rocfft_array_type_real
                                     : rocfft_array_type_hermitian_interleaved;
        rocfft_array_type out_t = type == rocfft_transform_type_real_forward
                                      ? rocfft_array_type_hermitian_interleaved
                                      : rocfft_array_type_real;
        NUSHT_FFT(rocfft_plan_description_set_data_layout(desc, in_t, out_t, nullptr, nullptr, 0,
                                                          nullptr, 0, 0, nullptr, 0));
    }
    rocfft_status st = rocfft_plan_create(&f.plan, place, type, prec, dim, lengths, batch, desc);
    rocfft_plan_description_destroy(desc);
    if (st != rocfft_status_success) {
        set_last_error("rocfft_plan_create", "failed");
        return NUSHT_EDEVICE;
    }
    NUSHT_FFT(rocfft_plan_get_work_buffer_size(f.plan, &f.work_bytes));
    NUSHT_FFT(rocfft_execution_info_create(&f.info));
    return NUSHT_OK;
}

// 1D batched transform with explicit strides and distances (in elements of the array types)
int make_fft_1d(FftPlan& f, rocfft_transform_type type, rocfft_precision prec, size_t len,
                size_t batch, size_t istride, size_t idist, size_t ostride, size_t odist,
                rocfft_result_placement place)
{
    rocfft_array_type in_t, out_t;
    if (type == rocfft_transform_type_real_forward) {
        in_t = rocfft_array_type_real;
        out_t = rocfft_array_type_hermitian_interleaved;
    } else if (type == rocfft_transform_type_real_inverse) {
        in_t = rocfft_array_type_hermitian_interleaved;
        out_t = rocfft_array_type_real;
    } else {
        in_t = out_t = rocfft_array_type_complex_interleaved;
    }
    rocfft_plan_description desc = nullptr;
    NUSHT_FFT(rocfft_plan_description_create(&desc));
    rocfft_status st = rocfft_plan_description_set_data_layout(
        desc, in_t, out_t, nullptr, nullptr, 1, &istride, idist, 1, &ostride, odist);
    if (st == rocfft_status_success)
        st = rocfft_plan_create(&f.plan, place, type, prec, 1, &len, batch, desc);
    rocfft_plan_description_destroy(desc);
    if (st != rocfft_status_success) {
        set_last_error("rocfft_plan_create", "failed (strided 1D)");
        return NUSHT_EDEVICE;
    }
    NUSHT_FFT(rocfft_plan_get_work_buffer_size(f.plan, &f.work_bytes));
    NUSHT_FFT(rocfft_execution_info_create(&f.info));
    return NUSHT_OK;
}

void free_fft(FftPlan& f)
{
    if (f.info) rocfft_execution_info_destroy(f.info);
    if (f.plan) rocfft_plan_destroy(f.plan);
    f.info = nullptr;
    f.plan = nullptr;
}

int ensure_ring_plans(nusht_plan_s* p);

}  // namespace

int create_fft_plans(nusht_plan_s* p)
{
    std::call_once(g_fft_once, [] { rocfft_setup(); });
    const nusht_geometry& g = p->g;
    const rocfft_precision prec =
        g.dtype == NUSHT_MIXED ? rocfft_precision_single : rocfft_precision_double;
    // Rows of the fine grid that any point window touches.  A point at theta has its first
    // tap in row ceil(theta n1 / (2 pi) - w/2) (mod n1), which for theta in [0, pi] lies in
    // [n1 - w/2, n1) or [0, floor(n1/2 - w/2) + 1]; a window spans the tile's kTile rows
    // plus w - 1.  Tile row n1 - kTile wraps into rows below kTile + w - 1.
    {
        const int last_tap = (int)std::floor(g.n1 / 2.0 - 0.5 * g.width) + 1;
        int ra = (last_tap / kTile + 1) * kTile + g.width - 1;
        int rb = kTile;
        if (ra + rb >= g.n1) {
            ra = g.n1;
            rb = 0;
        }
        p->fine_ra = ra;
        p->fine_rb = rb;
        // the spreading sweep: virtual tile rows [-1, vt_end) hold points, virtual rows
        // [-kTile, vrow_hi) are written (rb > 0: tile rows 0 .. ra/kTile - 1 and the w - 1 rows
        // after them; every row otherwise); segments sized for about 8192 waves
        const int nt1 = g.n1 / kTile;
        if (rb > 0) {
            p->band_vt_end = last_tap / kTile + 1;
            p->band_vrow_hi = ra;
        } else {
            p->band_vt_end = nt1 - 1;
            p->band_vrow_hi = g.n1 - kTile;
        }
        const long waves_per_row = (long)(g.n2 / p->band_w) / (64 / p->band_w);
        const long rows = p->band_vt_end + 1;
        long seg = waves_per_row * rows / 8192;
        p->band_seg_tiles = (int)std::max(1L, std::min(16L, seg));
    }
    const size_t fw = (size_t)g.n2 / 2 + 1;
    const size_t ncol = (size_t)g.mmax + 1;
    p->row_custom = rowfft_supported(g);
    p->theta_custom = thetafft_supported(g);
    if (p->theta_custom) {
        // twiddles of the fused theta pass: [2 n1] e^{2 pi i k / (2 n1)}, rounded once from
        // long double (the row kernels' table convention for an n1-point transform)
        const int n = 2 * g.n1;
        const bool f32 = g.dtype == NUSHT_MIXED;
        std::vector<double> tw(2 * (size_t)n);
        std::vector<float> twf(2 * (size_t)n);
        for (int k = 0; k < n; ++k) {
            const long double a = 2.0L * 3.14159265358979323846264338327950288L * k / n;
            tw[2 * k] = (double)cosl(a);
            tw[2 * k + 1] = (double)sinl(a);
            twf[2 * k] = (float)cosl(a);
            twf[2 * k + 1] = (float)sinl(a);
        }
        const size_t tb = 2 * (size_t)n * (f32 ? sizeof(float) : sizeof(double));
        if (hipMalloc(&p->thetatw, tb) != hipSuccess) {
            set_last_error("nusht_plan", "device allocation failed");
            return NUSHT_ENOMEM;
        }
        NUSHT_HIP(hipMemcpy(p->thetatw, f32 ? (const void*)twf.data() : (const void*)tw.data(),
                            tb, hipMemcpyHostToDevice));
    } else {
        NUSHT_TRY(make_fft_1d(p->fine_col_inv, rocfft_transform_type_complex_inverse, prec, g.n1,
                              ncol, 1, g.n1, 1, g.n1, rocfft_placement_inplace));
        NUSHT_TRY(make_fft_1d(p->fine_col_fwd, rocfft_transform_type_complex_forward, prec, g.n1,
                              ncol, 1, g.n1, 1, g.n1, rocfft_placement_inplace));
    }
    if (p->row_custom) {
        // twiddle table of the row kernels, rounded once from long double
        const int n2 = g.n2;
        const bool f32 = g.dtype == NUSHT_MIXED;
        std::vector<double> tw(2 * (size_t)n2);
        std::vector<float> twf(2 * (size_t)n2);
        for (int k = 0; k < n2; ++k) {
            const long double a = 2.0L * 3.14159265358979323846264338327950288L * k / n2;
            tw[2 * k] = (double)cosl(a);
            tw[2 * k + 1] = (double)sinl(a);
            twf[2 * k] = (float)cosl(a);
            twf[2 * k + 1] = (float)sinl(a);
        }
        const size_t tb = 2 * (size_t)n2 * (f32 ? sizeof(float) : sizeof(double));
        if (hipMalloc(&p->rowtw, tb) != hipSuccess) {
            set_last_error("nusht_plan", "device allocation failed");
            return NUSHT_ENOMEM;
        }
        NUSHT_HIP(hipMemcpy(p->rowtw, f32 ? (const void*)twf.data() : (const void*)tw.data(), tb,
                            hipMemcpyHostToDevice));
    } else {
        NUSHT_TRY(make_fft_1d(p->fine_rowa_c2r, rocfft_transform_type_real_inverse, prec, g.n2,
                              p->fine_ra, 1, fw, 1, g.n2, rocfft_placement_notinplace));
        NUSHT_TRY(make_fft_1d(p->fine_rowa_r2c, rocfft_transform_type_real_forward, prec, g.n2,
                              p->fine_ra, 1, g.n2, 1, fw, rocfft_placement_notinplace));
    }
    if (p->fine_rb > 0 && !p->row_custom) {
        NUSHT_TRY(make_fft_1d(p->fine_rowb_c2r, rocfft_transform_type_real_inverse, prec, g.n2,
                              p->fine_rb, 1, fw, 1, g.n2, rocfft_placement_notinplace));
        NUSHT_TRY(make_fft_1d(p->fine_rowb_r2c, rocfft_transform_type_real_forward, prec, g.n2,
                              p->fine_rb, 1, g.n2, 1, fw, rocfft_placement_notinplace));
    }
    if (g.dfs_mode == NUSHT_DFS_FUSED) {
        const size_t len = (size_t)g.ntorus;
        NUSHT_TRY(make_fft(p->theta_fwd, rocfft_transform_type_complex_forward, prec, 1, &len,
                           (size_t)g.mmax + 1, rocfft_placement_inplace));
        NUSHT_TRY(make_fft(p->theta_bwd, rocfft_transform_type_complex_inverse, prec, 1, &len,
                           (size_t)g.mmax + 1, rocfft_placement_inplace));
    } else {
        const size_t tl[2] = {(size_t)g.nphi, (size_t)g.ntorus};
        NUSHT_TRY(make_fft(p->torus_r2c, rocfft_transform_type_real_forward, prec, 2, tl, 1,
                           rocfft_placement_notinplace));
        NUSHT_TRY(make_fft(p->torus_c2r, rocfft_transform_type_real_inverse, prec, 2, tl, 1,
                           rocfft_placement_notinplace));
        NUSHT_TRY(ensure_ring_plans(p));
    }
    size_t work = 0;
    for (FftPlan* f : {&p->fine_col_inv, &p->fine_col_fwd, &p->fine_rowa_c2r, &p->fine_rowa_r2c,
                       &p->fine_rowb_c2r, &p->fine_rowb_r2c, &p->theta_fwd, &p->theta_bwd,
                       &p->torus_r2c, &p->torus_c2r, &p->ring_c2r, &p->ring_r2c})
        if (f->plan && f->work_bytes > work) work = f->work_bytes;
    if (work > p->fftwork_bytes) {
        if (p->fftwork) hipFree(p->fftwork);
        p->fftwork = nullptr;
        NUSHT_HIP(hipMalloc(&p->fftwork, work));
        p->fftwork_bytes = work;
    }
    return NUSHT_OK;
}

namespace {

int ensure_ring_plans(nusht_plan_s* p)
{
    if (p->ring_c2r.plan) return NUSHT_OK;
    const nusht_geometry& g = p->g;
    const size_t len = (size_t)g.nphi;
    NUSHT_TRY(make_fft(p->ring_c2r, rocfft_transform_type_real_inverse, rocfft_precision_double,
                       1, &len, (size_t)g.nrings, rocfft_placement_notinplace));
    NUSHT_TRY(make_fft(p->ring_r2c, rocfft_transform_type_real_forward, rocfft_precision_double,
                       1, &len, (size_t)g.nrings, rocfft_placement_notinplace));
    const size_t work = p->ring_c2r.work_bytes > p->ring_r2c.work_bytes ? p->ring_c2r.work_bytes
                                                                         : p->ring_r2c.work_bytes;
    if (work > p->fftwork_bytes) {
        if (p->fftwork) {
            NUSHT_HIP(hipDeviceSynchronize());
            hipFree(p->fftwork);
        }
        p->fftwork = nullptr;
        NUSHT_HIP(hipMalloc(&p->fftwork, work));
        p->fftwork_bytes = work;
    }
    return NUSHT_OK;
}

}  // namespace

void destroy_fft_plans(nusht_plan_s* p)
{
    for (FftPlan* f : {&p->fine_col_inv, &p->fine_col_fwd, &p->fine_rowa_c2r, &p->fine_rowa_r2c,
                       &p->fine_rowb_c2r, &p->fine_rowb_r2c, &p->theta_fwd, &p->theta_bwd,
                       &p->torus_r2c, &p->torus_c2r, &p->ring_c2r, &p->ring_r2c})
        free_fft(*f);
}

int fft_exec(nusht_plan_s* p, FftPlan& f, void* in, void* out, hipStream_t s)
{
    NUSHT_FFT(rocfft_execution_info_set_stream(f.info, s));
    if (f.work_bytes) NUSHT_FFT(rocfft_execution_info_set_work_buffer(f.info, p->fftwork, f.work_bytes));
    void* ib[1] = {in};
    void* ob[1] = {out};
    NUSHT_FFT(rocfft_execute(f.plan, ib, out ? ob : nullptr, f.info));
    return NUSHT_OK;
}

void stage_begin(nusht_plan_s* p, Stage st, hipStream_t s)
{
    if (!p->timing) return;
    hipEventRecord(p->ev[p->cur][st][0], s);
    p->ev_used[p->cur][st] = 1;
}

void stage_end(nusht_plan_s* p, Stage st, hipStream_t s)
{
    if (!p->timing) return;
    hipEventRecord(p->ev[p->cur][st][1], s);
}

namespace {

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        hipGetDevice(&prev);
        if (prev != dev) hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        int cur = -1;
        hipGetDevice(&cur);
        if (prev >= 0 && cur != prev) hipSetDevice(prev);
    }
};

// start of an execution call of the given kind: take the next timing slot
void begin_call(nusht_plan_s* p, int kind)
{
    if (!p->timing) return;
    p->cur = (int)(p->ncalls % nusht_plan_s::kTimingSlots);
    ++p->ncalls;
    p->slot_kind[p->cur] = kind;
    for (int i = 0; i < ST_COUNT; ++i) p->ev_used[p->cur][i] = 0;
}

inline char* bytes(void* v) { return reinterpret_cast<char*>(v); }

// fine grid (real) of map b and its half spectrum, in elements of the plan's precision
size_t fine_real_bytes(const nusht_plan_s* p) { return (size_t)p->g.n1 * p->g.n2 * fine_elem_bytes(p); }
// band spectrum [mmax+1][n1] of one map
size_t fine_band_bytes(const nusht_plan_s* p)
{
    return (size_t)(p->g.mmax + 1) * p->g.n1 * 2 * fine_elem_bytes(p);
}

// Band spectrum -> fine grid of one map (N(ii)): theta pass in place over the band (unless the
// fused theta pass has already written the band's window rows), transpose into the row
// spectrum of the window rows (p->W), phi pass into those rows of the grid.  Other rows of the
// grid are left untouched (no window reads them).
int fine_c2r(nusht_plan_s* p, char* band, char* real, hipStream_t s)
{
    const nusht_geometry& g = p->g;
    const size_t e = fine_elem_bytes(p);
    const size_t fw = (size_t)g.n2 / 2 + 1;
    char* rows = bytes(p->W);
    if (!p->theta_custom) NUSHT_TRY(fft_exec(p, p->fine_col_inv, band, nullptr, s));
    if (p->row_custom) {
        NUSHT_TRY(launch_band_to_rows(p, band, rows, g.mmax + 1, s));
        return launch_row_c2r(p, rows, g.mmax + 1, real, s);
    }
    NUSHT_TRY(launch_band_to_rows(p, band, rows, (int)fw, s));
    NUSHT_TRY(fft_exec(p, p->fine_rowa_c2r, rows, real, s));
    if (p->fine_rb > 0) {
        const size_t r0 = (size_t)g.n1 - p->fine_rb;
        NUSHT_TRY(fft_exec(p, p->fine_rowb_c2r, rows + r0 * fw * 2 * e, real + r0 * g.n2 * e, s));
    }
    return NUSHT_OK;
}

// Fine grid -> band spectrum of one map (N^H(ii)), reading only the window rows: phi pass
// over those rows into p->W, transpose into the band (zeros for the other rows), theta pass
// in place.  With the fused theta pass only the window rows of the band are written and its
// theta pass runs later, with the deconvolution.
int fine_r2c(nusht_plan_s* p, char* real, char* band, hipStream_t s)
{
    const nusht_geometry& g = p->g;
    const size_t e = fine_elem_bytes(p);
    const size_t fw = (size_t)g.n2 / 2 + 1;
    char* rows = bytes(p->W);
    if (p->row_custom) {
        NUSHT_TRY(launch_row_r2c(p, real, rows, g.mmax + 1, s));
        NUSHT_TRY(launch_rows_to_band(p, rows, g.mmax + 1, band, s, p->theta_custom));
        if (p->theta_custom) return NUSHT_OK;
        return fft_exec(p, p->fine_col_fwd, band, nullptr, s);
    }
    NUSHT_TRY(fft_exec(p, p->fine_rowa_r2c, real, rows, s));
    if (p->fine_rb > 0) {
        const size_t r0 = (size_t)g.n1 - p->fine_rb;
        NUSHT_TRY(fft_exec(p, p->fine_rowb_r2c, real + r0 * g.n2 * e, rows + r0 * fw * 2 * e, s));
    }
    NUSHT_TRY(launch_rows_to_band(p, rows, (int)fw, band, s));
    NUSHT_TRY(fft_exec(p, p->fine_col_fwd, band, nullptr, s));
    return NUSHT_OK;
}

// S (Legendre + per-ring phi-FFT) of the paper composition into ring maps [b][N_r][N_phi];
// spin > 0: the maps are the (Q, U) pairs of nmaps / 2 spin-weighted fields
int ring_synthesis_into(nusht_plan_s* p, const double* alm, double* ring, void* G, int nmaps,
                        hipStream_t s, int spin = 0)
{
    const nusht_geometry& g = p->g;
    stage_begin(p, ST_LEGENDRE, s);
    if (spin)
        NUSHT_TRY(launch_spin_synth(p, spin, alm, G, nmaps / 2, 0, s, false));
    else
        NUSHT_TRY(launch_legendre_synth(p, alm, G, nmaps, 0, 0, s));
    NUSHT_TRY(launch_zero_nyquist_rows(p, reinterpret_cast<double*>(G), nmaps, s));
    stage_end(p, ST_LEGENDRE, s);
    stage_begin(p, ST_RING_FFT, s);
    const size_t gstride = (size_t)g.nrings * (g.nphi / 2 + 1) * 16;
    const size_t rstride = (size_t)g.nrings * g.nphi * 8;
    for (int b = 0; b < nmaps; ++b)
        NUSHT_TRY(fft_exec(p, p->ring_c2r, bytes(G) + b * gstride, bytes(ring) + b * rstride, s));
    stage_end(p, ST_RING_FFT, s);
    return NUSHT_OK;
}

// torus spectrum (fused: doubled theta-columns [b][m][t] transformed over t; paper: 2D R2C
// of the doubled map) into X, for maps [0, nmaps)
// spin > 0: the nmaps maps are the (Q, U) pairs of nmaps / 2 spin-weighted fields, whose
// columns come from the Wigner-d step and whose doubling carries (-1)^spin
int synthesis_to_fine(nusht_plan_s* p, const double* alm, int nmaps, hipStream_t s, void** fine_out,
                      int spin = 0)
{
    const nusht_geometry& g = p->g;
    const int f32 = g.dtype == NUSHT_MIXED;
    const size_t e = fine_elem_bytes(p);
    if (g.dfs_mode == NUSHT_DFS_FUSED) {
        stage_begin(p, ST_LEGENDRE, s);
        if (spin)
            NUSHT_TRY(launch_spin_synth(p, spin, alm, p->X, nmaps / 2, f32, s));
        else
            NUSHT_TRY(launch_legendre_synth(p, alm, p->X, nmaps, 1, f32, s));
        stage_end(p, ST_LEGENDRE, s);
        stage_begin(p, ST_TORUS_FFT, s);
        const size_t cstride = (size_t)(g.mmax + 1) * g.ntorus * 2 * e;
        for (int b = 0; b < nmaps; ++b)
            NUSHT_TRY(fft_exec(p, p->theta_fwd, bytes(p->X) + b * cstride, nullptr, s));
        stage_end(p, ST_TORUS_FFT, s);
        stage_begin(p, ST_DECONV, s);
        if (p->theta_custom)
            NUSHT_TRY(launch_theta_inv(p, p->X, p->Y, nmaps, s));
        else
            NUSHT_TRY(launch_deconv_pad(p, p->X, p->Y, nmaps, 1, f32, s));
        stage_end(p, ST_DECONV, s);
        stage_begin(p, ST_FINE_FFT, s);
        for (int b = 0; b < nmaps; ++b)
            NUSHT_TRY(fine_c2r(p, bytes(p->Y) + b * fine_band_bytes(p),
                               bytes(p->X) + b * fine_real_bytes(p), s));
        stage_end(p, ST_FINE_FFT, s);
        *fine_out = p->X;
    } else {
        NUSHT_TRY(ring_synthesis_into(p, alm, reinterpret_cast<double*>(p->Y), p->X, nmaps, s,
                                      spin));
        stage_begin(p, ST_DOUBLE, s);
        NUSHT_TRY(launch_double(p, reinterpret_cast<const double*>(p->Y), p->X, nmaps, f32, s,
                                (spin & 1) ? -1.0 : 1.0));
        stage_end(p, ST_DOUBLE, s);
        stage_begin(p, ST_TORUS_FFT, s);
        const size_t tstride = (size_t)g.ntorus * g.nphi * e;
        const size_t sstride = (size_t)g.ntorus * (g.nphi / 2 + 1) * 2 * e;
        for (int b = 0; b < nmaps; ++b)
            NUSHT_TRY(fft_exec(p, p->torus_r2c, bytes(p->X) + b * tstride,
                               bytes(p->Y) + b * sstride, s));
        stage_end(p, ST_TORUS_FFT, s);
        stage_begin(p, ST_DECONV, s);
        NUSHT_TRY(launch_deconv_pad(p, p->Y, p->X, nmaps, 0, f32, s));
        stage_end(p, ST_DECONV, s);
        stage_begin(p, ST_FINE_FFT, s);
        for (int b = 0; b < nmaps; ++b)
            NUSHT_TRY(fine_c2r(p, bytes(p->X) + b * fine_band_bytes(p),
                               bytes(p->Y) + b * fine_real_bytes(p), s));
        stage_end(p, ST_FINE_FFT, s);
        *fine_out = p->Y;
    }
    return NUSHT_OK;
}

// the spin-weighted calls: 1 <= spin <= min(lmax, NUSHT_MAX_SPIN) and the exponent-range limit
}  // namespace

int check_spin(nusht_plan_s* p, int spin, const char* who)
{
    if (spin < 1 || spin > p->g.lmax || spin > NUSHT_MAX_SPIN) {
        set_last_error(who, "spin must satisfy 1 <= spin <= min(lmax, NUSHT_MAX_SPIN)");
        return NUSHT_EINVAL;
    }
    // The two Wigner-d functions of a ring share one binary exponent; at the ring next to a
    // pole, d^l_{m,-s} starts tan^(2 min(m, s))(theta_1 / 2) times d^l_{m,+s}.  Below 2^-800
    // it could leave the FP64 range and stay zero for every l, so such spins are refused.
    const double t1 = std::tan(0.5 * M_PI / (double)(p->g.nrings - 1));
    if (2.0 * spin * -std::log2(t1) > 800.0) {
        set_last_error(who, "spin too high for this ring grid (2 s log2(1/tan(theta_1/2)) > 800)");
        return NUSHT_EINVAL;
    }
    return NUSHT_OK;
}

namespace {

int check_exec(nusht_plan_s* p, const void* a, const void* b, int nmaps)
{
    if (!p) {
        set_last_error("nusht", "null plan");
        return NUSHT_EINVAL;
    }
    if (!a || !b || nmaps < 1) {
        set_last_error("nusht", "null buffer or nmaps < 1");
        return NUSHT_EINVAL;
    }
    return NUSHT_OK;
}

}  // namespace
}  // namespace nusht

using namespace nusht;

extern "C" {

int nusht_synthesis(nusht_plan_t p, const double* alm, double* map, int nmaps, void* stream)
{
    NUSHT_TRY(check_exec(p, alm, map, nmaps));
    DeviceGuard dg(p->device);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    NUSHT_TRY(ensure_capacity(p, nmaps));
    begin_call(p, NUSHT_CALL_SYNTHESIS);
    void* fine = nullptr;
    NUSHT_TRY(synthesis_to_fine(p, alm, nmaps, s, &fine));
    stage_begin(p, ST_POINTS, s);
    if (p->g.dtype == NUSHT_MIXED)
        NUSHT_TRY(interp_f32(p, reinterpret_cast<const float*>(fine), map, nmaps, s));
    else
        NUSHT_TRY(interp_f64(p, reinterpret_cast<const double*>(fine), map, nmaps, s));
    stage_end(p, ST_POINTS, s);
    return NUSHT_OK;
}

int nusht_synthesis_deriv(nusht_plan_t p, const double* alm, double* map, double* dtheta,
                          double* dphi, int nmaps, void* stream)
{
    NUSHT_TRY(check_exec(p, alm, map, nmaps));
    if (!dtheta || !dphi) return NUSHT_EINVAL;
    if (p->g.dtype != NUSHT_F64) {
        set_last_error("nusht_synthesis_deriv", "needs an FP64 plan");
        return NUSHT_EPRECISION;
    }
    DeviceGuard dg(p->device);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    NUSHT_TRY(ensure_capacity(p, nmaps));
    begin_call(p, NUSHT_CALL_SYNTHESIS_DERIV);
    void* fine = nullptr;
    NUSHT_TRY(synthesis_to_fine(p, alm, nmaps, s, &fine));
    stage_begin(p, ST_POINTS, s);
    NUSHT_TRY(launch_interp_deriv(p, reinterpret_cast<const double*>(fine), map, dtheta, dphi,
                                  nmaps, s));
    stage_end(p, ST_POINTS, s);
    return NUSHT_OK;
}

int nusht_synthesis_spin_deriv(nusht_plan_t p, int spin, const double* alm, double* map,
                               double* dtheta, double* dphi, int nfields, void* stream)
{
    NUSHT_TRY(check_exec(p, alm, map, nfields));
    NUSHT_TRY(check_spin(p, spin, "nusht_synthesis_spin_deriv"));
    if (!dtheta || !dphi) return NUSHT_EINVAL;
    if (p->g.dtype != NUSHT_F64) {
        set_last_error("nusht_synthesis_spin_deriv", "needs an FP64 plan");
        return NUSHT_EPRECISION;
    }
    DeviceGuard dg(p->device);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    NUSHT_TRY(ensure_capacity(p, 2 * nfields));
    begin_call(p, NUSHT_CALL_SYNTHESIS_DERIV);
    void* fine = nullptr;
    NUSHT_TRY(synthesis_to_fine(p, alm, 2 * nfields, s, &fine, spin));
    stage_begin(p, ST_POINTS, s);
    NUSHT_TRY(launch_interp_deriv(p, reinterpret_cast<const double*>(fine), map, dtheta, dphi,
                                  2 * nfields, s));
    stage_end(p, ST_POINTS, s);
    return NUSHT_OK;
}

}  // extern "C"

namespace nusht {
namespace {

// N^H, then the fused or paper-mode S^H; spin > 0: nmaps / 2 spin-weighted fields
int adjoint_impl(nusht_plan_s* p, const double* map, double* alm, int nmaps, hipStream_t s,
                 int spin)
{
    const nusht_geometry& g = p->g;
    const int f32 = g.dtype == NUSHT_MIXED;
    const size_t e = fine_elem_bytes(p);
    // N^H (i): spreading of each group of maps straight onto their fine grids (window rows)
    stage_begin(p, ST_POINTS, s);
    for (int b = 0; b < nmaps;) {
        const int mb = group_width(nmaps, b);
        char* fine = bytes(p->X) + b * fine_real_bytes(p);
        if (f32)
            NUSHT_TRY(spread_group_f32(p, map + b * g.npts, reinterpret_cast<float*>(fine), mb, s));
        else
            NUSHT_TRY(spread_group_f64(p, map + b * g.npts, reinterpret_cast<double*>(fine), mb, s));
        b += mb;
    }
    stage_end(p, ST_POINTS, s);
    // N^H (ii): fine-grid R2C
    stage_begin(p, ST_FINE_FFT, s);
    for (int b = 0; b < nmaps; ++b)
        NUSHT_TRY(fine_r2c(p, bytes(p->X) + b * fine_real_bytes(p),
                           bytes(p->Y) + b * fine_band_bytes(p), s));
    stage_end(p, ST_FINE_FFT, s);
    if (g.dfs_mode == NUSHT_DFS_FUSED) {
        stage_begin(p, ST_DECONV, s);
        if (p->theta_custom)
            NUSHT_TRY(launch_theta_fwd(p, p->Y, p->X, nmaps, s));
        else
            NUSHT_TRY(launch_deconv_trunc(p, p->Y, p->X, nmaps, 1, f32, s));
        stage_end(p, ST_DECONV, s);
        stage_begin(p, ST_TORUS_FFT, s);
        const size_t cstride = (size_t)(g.mmax + 1) * g.ntorus * 2 * e;
        for (int b = 0; b < nmaps; ++b)
            NUSHT_TRY(fft_exec(p, p->theta_bwd, bytes(p->X) + b * cstride, nullptr, s));
        stage_end(p, ST_TORUS_FFT, s);
        stage_begin(p, ST_LEGENDRE, s);
        if (spin)
            NUSHT_TRY(launch_spin_adjoint(p, spin, p->X, alm, nmaps / 2, f32, s));
        else
            NUSHT_TRY(launch_legendre_adjoint(p, p->X, alm, nmaps, 1, f32, s));
        stage_end(p, ST_LEGENDRE, s);
    } else {
        stage_begin(p, ST_DECONV, s);
        NUSHT_TRY(launch_deconv_trunc(p, p->Y, p->X, nmaps, 0, f32, s));
        stage_end(p, ST_DECONV, s);
        stage_begin(p, ST_TORUS_FFT, s);
        const size_t tstride = (size_t)g.ntorus * g.nphi * e;
        const size_t sstride = (size_t)g.ntorus * (g.nphi / 2 + 1) * 2 * e;
        for (int b = 0; b < nmaps; ++b)
            NUSHT_TRY(fft_exec(p, p->torus_c2r, bytes(p->X) + b * sstride,
                               bytes(p->Y) + b * tstride, s));
        stage_end(p, ST_TORUS_FFT, s);
        stage_begin(p, ST_DOUBLE, s);
        NUSHT_TRY(launch_fold(p, p->Y, reinterpret_cast<double*>(p->X), nmaps, f32, s,
                              (spin & 1) ? -1.0 : 1.0));
        stage_end(p, ST_DOUBLE, s);
        stage_begin(p, ST_RING_FFT, s);
        const size_t rstride = (size_t)g.nrings * g.nphi * 8;
        const size_t gstride = (size_t)g.nrings * (g.nphi / 2 + 1) * 16;
        for (int b = 0; b < nmaps; ++b)
            NUSHT_TRY(fft_exec(p, p->ring_r2c, bytes(p->X) + b * rstride,
                               bytes(p->Y) + b * gstride, s));
        stage_end(p, ST_RING_FFT, s);
        stage_begin(p, ST_LEGENDRE, s);
        if (spin)
            NUSHT_TRY(launch_spin_adjoint(p, spin, p->Y, alm, nmaps / 2, 0, s, false));
        else
            NUSHT_TRY(launch_legendre_adjoint(p, p->Y, alm, nmaps, 0, 0, s));
        stage_end(p, ST_LEGENDRE, s);
    }
    return NUSHT_OK;
}

}  // namespace
}  // namespace nusht

extern "C" {

int nusht_adjoint(nusht_plan_t p, const double* map, double* alm, int nmaps, void* stream)
{
    NUSHT_TRY(check_exec(p, map, alm, nmaps));
    DeviceGuard dg(p->device);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    NUSHT_TRY(ensure_capacity(p, nmaps));
    begin_call(p, NUSHT_CALL_ADJOINT);
    return adjoint_impl(p, map, alm, nmaps, s, 0);
}

int nusht_synthesis_spin(nusht_plan_t p, int spin, const double* alm, double* map, int nfields,
                         void* stream)
{
    NUSHT_TRY(check_exec(p, alm, map, nfields));
    NUSHT_TRY(check_spin(p, spin, "nusht_synthesis_spin"));
    DeviceGuard dg(p->device);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    NUSHT_TRY(ensure_capacity(p, 2 * nfields));
    begin_call(p, NUSHT_CALL_SPIN_SYNTHESIS);
    void* fine = nullptr;
    NUSHT_TRY(synthesis_to_fine(p, alm, 2 * nfields, s, &fine, spin));
    stage_begin(p, ST_POINTS, s);
    if (p->g.dtype == NUSHT_MIXED)
        NUSHT_TRY(interp_f32(p, reinterpret_cast<const float*>(fine), map, 2 * nfields, s));
    else
        NUSHT_TRY(interp_f64(p, reinterpret_cast<const double*>(fine), map, 2 * nfields, s));
    stage_end(p, ST_POINTS, s);
    return NUSHT_OK;
}

int nusht_adjoint_spin(nusht_plan_t p, int spin, const double* map, double* alm, int nfields,
                       void* stream)
{
    NUSHT_TRY(check_exec(p, map, alm, nfields));
    NUSHT_TRY(check_spin(p, spin, "nusht_adjoint_spin"));
    DeviceGuard dg(p->device);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    NUSHT_TRY(ensure_capacity(p, 2 * nfields));
    begin_call(p, NUSHT_CALL_SPIN_ADJOINT);
    return adjoint_impl(p, map, alm, 2 * nfields, s, spin);
}

int nusht_ring_synthesis(nusht_plan_t p, const double* alm, double* ring, int nmaps, void* stream)
{
    NUSHT_TRY(check_exec(p, alm, ring, nmaps));
    DeviceGuard dg(p->device);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    NUSHT_TRY(ensure_ring_plans(p));
    NUSHT_TRY(ensure_capacity(p, nmaps));
    begin_call(p, NUSHT_CALL_RING);
    return ring_synthesis_into(p, alm, ring, p->X, nmaps, s);
}

int nusht_ring_adjoint(nusht_plan_t p, const double* ring, double* alm, int nmaps, void* stream)
{
    NUSHT_TRY(check_exec(p, ring, alm, nmaps));
    DeviceGuard dg(p->device);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    NUSHT_TRY(ensure_ring_plans(p));
    NUSHT_TRY(ensure_capacity(p, nmaps));
    begin_call(p, NUSHT_CALL_RING);
    const nusht_geometry& g = p->g;
    const size_t rstride = (size_t)g.nrings * g.nphi * 8;
    const size_t gstride = (size_t)g.nrings * (g.nphi / 2 + 1) * 16;
    // rocFFT may overwrite the input of an out-of-place transform: work on a copy
    NUSHT_HIP(hipMemcpyAsync(p->X, ring, rstride * nmaps, hipMemcpyDeviceToDevice, s));
    stage_begin(p, ST_RING_FFT, s);
    for (int b = 0; b < nmaps; ++b)
        NUSHT_TRY(fft_exec(p, p->ring_r2c, bytes(p->X) + b * rstride, bytes(p->Y) + b * gstride, s));
    stage_end(p, ST_RING_FFT, s);
    stage_begin(p, ST_LEGENDRE, s);
    NUSHT_TRY(launch_legendre_adjoint(p, p->Y, alm, nmaps, 0, 0, s));
    stage_end(p, ST_LEGENDRE, s);
    return NUSHT_OK;
}

static const char* kStageNames[ST_COUNT] = {"legendre", "ring_fft", "double_fold", "torus_fft",
                                            "deconv", "fine_fft", "points"};

int nusht_stage_times(nusht_plan_t p, double* ms, const char** names, int maxn)
{
    if (!p || !ms || maxn < 0) return NUSHT_EINVAL;
    if (!p->timing || p->ncalls == 0) return 0;
    const int c = p->cur;
    int n = 0;
    for (int i = 0; i < ST_COUNT && n < maxn; ++i) {
        float t = 0.0f;
        if (p->ev_used[c][i]) {
            if (hipEventSynchronize(p->ev[c][i][1]) != hipSuccess ||
                hipEventElapsedTime(&t, p->ev[c][i][0], p->ev[c][i][1]) != hipSuccess)
                t = -1.0f;
        }
        ms[n] = p->ev_used[c][i] ? (double)t : 0.0;
        if (names) names[n] = kStageNames[i];
        ++n;
    }
    return n;
}

int nusht_stage_stats(nusht_plan_t p, int kind, double* ms, int* ncalls, const char** names,
                      int maxn)
{
    if (!p || !ms || maxn < 0) return NUSHT_EINVAL;
    NUSHT_TRY(check_device_status(p));
    if (!p->timing) return 0;
    const int nslot = (int)(p->ncalls < nusht_plan_s::kTimingSlots ? p->ncalls
                                                                   : nusht_plan_s::kTimingSlots);
    int n = 0;
    for (int i = 0; i < ST_COUNT && n < maxn; ++i) {
        double sum = 0.0;
        int cnt = 0;
        for (int c = 0; c < nslot; ++c) {
            if (p->slot_kind[c] != kind || !p->ev_used[c][i]) continue;
            float t = 0.0f;
            if (hipEventSynchronize(p->ev[c][i][1]) != hipSuccess ||
                hipEventElapsedTime(&t, p->ev[c][i][0], p->ev[c][i][1]) != hipSuccess) {
                set_last_error("nusht_stage_stats", "event query failed");
                return NUSHT_EDEVICE;
            }
            sum += t;
            ++cnt;
        }
        ms[n] = cnt ? sum / cnt : 0.0;
        if (ncalls) ncalls[n] = cnt;
        if (names) names[n] = kStageNames[i];
        ++n;
    }
    return n;
}

void nusht_stage_reset(nusht_plan_t p)
{
    if (p) p->ncalls = 0;
}

}  // extern "C"

// Internal declarations of the nusht library (gfx950).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <rocfft/rocfft.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/nusht.h"

namespace nusht {

// Side of the square tiles the points are binned into on the fine grid.  Every tile window
// (tile + w - 1 cells a side) must fit in LDS for the interpolation; w <= 16 keeps a point's
// taps inside the next tile row, which the spreading sweep's segment overlap relies on.
constexpr int kTile = 32;
constexpr int kMaxWidth = 16;
// zero entries after the recurrence table, so that a chunk of l values can be loaded whole
constexpr int kRecPad = 64;
constexpr int kMinWidth = 2;
// bits of a plan's device error word
constexpr int kErrAdjWait = 1;  // a Legendre-adjoint slot wait reached its bound

// Reads the plan's device error word (synchronises the plan's device); NUSHT_EDEVICE if any
// kernel has set it.
int check_device_status(nusht_plan_s* p);

// Status that keeps the first failing HIP/rocFFT call for diagnostics.
struct Err {
    int code = NUSHT_OK;
};

#define NUSHT_HIP(call)                                                   \
    do {                                                                  \
        hipError_t e_ = (call);                                           \
        if (e_ != hipSuccess) {                                           \
            ::nusht::set_last_error(#call, hipGetErrorString(e_));        \
            return e_ == hipErrorOutOfMemory ? NUSHT_ENOMEM : NUSHT_EDEVICE; \
        }                                                                 \
    } while (0)

#define NUSHT_FFT(call)                                                   \
    do {                                                                  \
        rocfft_status s_ = (call);                                        \
        if (s_ != rocfft_status_success) {                                \
            ::nusht::set_last_error(#call, "rocfft failure");             \
            return NUSHT_EDEVICE;                                         \
        }                                                                 \
    } while (0)

#define NUSHT_TRY(expr)             \
    do {                            \
        int r_ = (expr);            \
        if (r_ != NUSHT_OK) return r_; \
    } while (0)

void set_last_error(const char* what, const char* why);

// One rocFFT transform with its execution info (stream and work buffer bound per call).
struct FftPlan {
    rocfft_plan plan = nullptr;
    rocfft_execution_info info = nullptr;
    size_t work_bytes = 0;
};

// Stage identifiers for the optional per-stage timing.
enum Stage {
    ST_LEGENDRE = 0,  // a1 / b7
    ST_RING_FFT,      // a2 / b6 (paper mode)
    ST_DOUBLE,        // a3 / b5
    ST_TORUS_FFT,     // a4 / b4
    ST_DECONV,        // a5 / b3
    ST_FINE_FFT,      // a6 / b2
    ST_POINTS,        // a7 / b1 (interpolation or spreading)
    ST_COUNT
};

}  // namespace nusht

struct nusht_plan_s {
    nusht_geometry g{};
    double eps = 0;
    int device = 0;
    hipStream_t plan_stream = nullptr;
    // Second stream of the Legendre synthesis (default priority): its plain-range instance runs
    // there beside the scaled-range instance on the call's stream; fork / join events.
    hipStream_t side = nullptr;
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;

    // Legendre tables (host-computed, FP64).
    double2* rec = nullptr;      // [nalm]: (a_lm, a_lm * b_lm) of the recurrence, l >= m+1
    double* cm_mant = nullptr;   // [mmax+1]: lam_mm prefactor mantissa, sign (-1)^m included
    int* cm_exp = nullptr;       // [mmax+1]: its power-of-two exponent
    int* jlive = nullptr;        // [mmax+1]: first ring pair with any lam_lm above 2^-300
    int* jscale = nullptr;       // [mmax+1]: first ring pair with lam_mm above 2^-190
    std::vector<int> jlive_host;

    // Wigner-d tables of the spin-weighted Legendre step (spin.hip), for spin spin_s (0: none):
    // (alpha, c_p, c_q, gamma) of the step to (l, m) and the start constant per m.
    int spin_s = 0;
    double4* spin_rec = nullptr;  // [nalm + kRecPad]
    double* spin_km = nullptr;    // [mmax+1] mantissa
    int* spin_ke = nullptr;       // [mmax+1] power-of-two exponent
    int* spin_jlive = nullptr;    // [mmax+1] first ring pair with any value above 2^-300

    // Deconvolution factors (include the FFT normalisation of the torus transform).
    double* dec1 = nullptr;      // [lmax+1], indexed by |kappa|
    double* dec2 = nullptr;      // [mmax+1], indexed by mu
    float* dec1f = nullptr;
    float* dec2f = nullptr;

    // Points binned into tiles ("slots" are the tiles that hold points, in tile order).
    double* sth = nullptr;       // [npts] theta, sorted by tile
    double* sph = nullptr;       // [npts] phi mod 2 pi, sorted by tile
    int* perm = nullptr;         // [npts] user index of each sorted point
    int* iperm = nullptr;        // [npts] sorted index of each user point (inverse of perm)
    int* slot_off = nullptr;     // [nslots+1] first sorted point of each slot
    int* slot_tile = nullptr;    // [nslots] tile id of each slot
    int* tile_slot = nullptr;    // [ntiles] slot of each tile or -1
    // Records of the spreading sweep: the fine columns are cut into bands of band_w columns
    // (band_w >= w); every point has a record in its own band and one in the next band when
    // its taps reach it, sorted by (band, tile row, row); boff[band * nt1 + tile row] is the
    // first record of that band and tile row.  Records hold the first-tap row and the column
    // relative to the band, the caller's point index and the two tap offsets in the plan's
    // precision (BandRec<float> or BandRec<double>).
    void* brec = nullptr;
    int64_t nrec = 0;
    int* boff = nullptr;         // [n2 / band_w * nt1 + 1]
    int band_w = 0;
    // Rows of the spreading sweep on a virtual axis (tile row nt1 - 1 is tile row -1): tile
    // rows [-1, band_vt_end) can hold points, rows [-kTile, band_vrow_hi) are written, in
    // segments of band_seg_tiles tile rows.
    int band_vt_end = 0, band_vrow_hi = 0, band_seg_tiles = 1;
    int nslots = 0;
    int nt1 = 0, nt2 = 0;        // tiles per fine-grid axis
    int* dflag = nullptr;        // device error flag used by plan validation
    int* dstatus = nullptr;      // device error word of the execution kernels (kErr* bits),
                                 // sticky until the plan is destroyed

    // Scratch, grown to the largest batch seen.  Two ping-pong regions and one for the
    // spread subgrids.
    int bcap = 0;
    void* X = nullptr;
    size_t Xbytes = 0;
    void* Y = nullptr;
    size_t Ybytes = 0;
    void* W = nullptr;           // one map's fine row spectrum [n1][n2/2+1]
    size_t Wbytes = 0;
    double* V = nullptr;         // point scratch [npts][4]: packed point values of one group
    void* Z = nullptr;           // tile subgrids of the wide-kernel spreading [nslots][P][P][4]
    size_t Zbytes = 0;
    void* fftwork = nullptr;
    size_t fftwork_bytes = 0;
    double* red = nullptr;       // small reduction scratch for the CG solve
    size_t redbytes = 0;
    // ES taps: polynomial coefficients [(w + 1) * w] (s^k of tap a at k * w + a) in FP64 and
    // FP32, or null when the taps are formed from sqrt and exp (option, or fit not accurate)
    int es_eval = 0;
    double es_poly_dev = 0.0;
    double* es_coef = nullptr;
    float* es_coeff = nullptr;
    // deterministic plans: the Legendre adjoint's per-pair-chunk partial sums
    int deterministic = 0;
    double* adj_part = nullptr;
    size_t adj_part_bytes = 0;

    // rocFFT plans (all per map; executed once per map of a batch).
    nusht::FftPlan ring_c2r, ring_r2c;      // 1D over phi, batch N_r, FP64
    nusht::FftPlan torus_r2c, torus_c2r;    // 2D N_t x N_phi (paper mode)
    nusht::FftPlan theta_fwd, theta_bwd;    // 1D C2C over N_t, batch mmax+1 (fused mode)
    // Fine grid n1 x n2 (real) <-> n1 x (n2/2+1) (half spectrum), split into its two passes
    // and pruned: the theta pass runs only over the mmax+1 columns that carry the band
    // limit, the phi pass only over the rows [0, fine_ra) and [n1 - fine_rb, n1) that the
    // point windows touch (theta in [0, pi] covers half of the doubled theta circle).  The
    // band columns are stored transposed, [mu][i] ("band spectrum"), so that the theta pass
    // is a contiguous batched FFT; an LDS-tiled transpose links them to the row spectrum.
    nusht::FftPlan fine_col_inv, fine_col_fwd;  // 1D C2C over n1, batch mmax+1, contiguous
    nusht::FftPlan fine_rowa_c2r, fine_rowa_r2c;  // 1D over n2, batch fine_ra
    nusht::FftPlan fine_rowb_c2r, fine_rowb_r2c;  // 1D over n2, batch fine_rb (may be empty)
    int fine_ra = 0, fine_rb = 0;
    // n2 / 2 = 2^K or 5 2^K: the phi pass runs in the library's own row kernels (rowfft.hip),
    // on row spectra of width mmax + 1 (no zero columns), instead of the rocFFT row plans.
    bool row_custom = false;
    void* rowtw = nullptr;  // [n2] e^{2 pi i k / n2} in the plan's FFT precision
    // Fused mode with n1 = 2^K or 5 2^K up to 16384: the theta pass and the deconvolution run
    // as one kernel per direction (rowfft.hip) instead of the rocFFT column plans and the pad /
    // truncate kernels.
    bool theta_custom = false;
    void* thetatw = nullptr;  // [2 n1] e^{2 pi i k / (2 n1)} in the plan's FFT precision

    // Timing.
    // Timing: every execution call takes the next slot of a ring of kTimingSlots slots, each
    // with one event pair per stage; nusht_stage_stats averages the calls of one kind.
    static constexpr int kTimingSlots = 64;
    int timing = 0;
    hipEvent_t ev[kTimingSlots][nusht::ST_COUNT][2]{};
    unsigned char ev_used[kTimingSlots][nusht::ST_COUNT]{};
    int slot_kind[kTimingSlots]{};
    int64_t ncalls = 0;   // calls since the last reset
    int cur = 0;          // slot of the current call
};

namespace nusht {

// Width of the column bands of the spreading kernel (one band per lane group of a wave): the
// taps of a point reach at most w - 1 columns past its first tap, so one band to the left holds
// every point that reaches a band, and the group's lanes hold the w row taps of a point.
inline int band_width_for(int w) { return w <= 8 ? 8 : 16; }

// A record of the spreading sweep: rc = first-tap row | (column relative to the band + 32) << 16,
// src = the caller's point index, s1 / s2 = tap offsets as s = 2 d - w + 1 in (-1, 1]
template <typename T>
struct BandRec {
    int rc;
    int src;
    T s1, s2;
};

// Maps are processed by the point kernels in groups of four, the remainder one by one.
inline int group_width(int nmaps, int b) { return (nmaps - b) >= 4 ? 4 : 1; }

// Spreading strategy: the band sweep for every FP32 (mixed-precision) kernel, for FP64 kernels
// of width <= 8 and for deterministic plans; tile subgrids with LDS atomics and a halo pass for
// wider FP64 kernels (whose band sweep runs one map per pass).
inline bool spread_uses_tiles(const nusht_plan_s* p)
{
    return p->g.dtype == NUSHT_F64 && p->g.width > 8 && !p->deterministic;
}

// ---- geometry (plan.hip) ----
int compute_geometry(int lmax, int mmax, double eps, int dtype, const nusht_plan_opts* opts,
                     nusht_geometry* g);
int ensure_capacity(nusht_plan_s* p, int nmaps);
size_t fine_elem_bytes(const nusht_plan_s* p);

// ---- FFT helpers (transform.hip) ----
int fft_exec(nusht_plan_s* p, FftPlan& f, void* in, void* out, hipStream_t s);

// ---- timing helpers (transform.hip) ----
void stage_begin(nusht_plan_s* p, Stage st, hipStream_t s);
void stage_end(nusht_plan_s* p, Stage st, hipStream_t s);

// ---- Legendre (legendre.hip) ----
// Output layouts of the synthesis: PAPER writes G[b][j][m] (rows of N_phi/2+1 complex, the
// ring FFT's input); FUSED writes the doubled column Gt[b][m][t], t < N_t.
int launch_legendre_synth(const nusht_plan_s* p, const double* alm, void* out, int nmaps,
                          int fused, int out_f32, hipStream_t s);
// ring pairs per lane of the synthesis' plain instance
int synth_pairs_per_lane(int npairs);
int synth_scaled_pairs_per_lane(int npairs);
// adjoint into alm [nmaps][nalm] (complex128), which it zeroes and then accumulates into
int launch_legendre_adjoint(nusht_plan_s* p, const void* in, double* alm, int nmaps,
                            int fused, int in_f32, hipStream_t s);

// ---- DFS glue (dfs.hip) ----
// ---- spin-weighted Legendre step (spin.hip) ----
// tables for the given spin (rebuilt when it changes); nfields fields = 2 nfields maps (Q, U)
int ensure_spin_tables(nusht_plan_s* p, int spin);
// host check of a spin argument (range, and the shared-exponent limit of the ring grid)
int check_spin(nusht_plan_s* p, int spin, const char* who);
// fused: the doubled theta-columns [map][m][t]; otherwise the ring layout [map][j][m] with rows
// of N_phi/2 + 1 (FP64) of the paper composition
int launch_spin_synth(nusht_plan_s* p, int spin, const double* alm, void* out, int nfields,
                      int out_f32, hipStream_t s, bool fused = true);
int launch_spin_adjoint(nusht_plan_s* p, int spin, const void* in, double* alm, int nfields,
                        int in_f32, hipStream_t s, bool fused = true);
int launch_zero_nyquist_rows(const nusht_plan_s* p, double* G, int nmaps, hipStream_t s);
// sgn: sign of the doubled half ((-1)^s for spin-s components, 1 otherwise)
int launch_double(const nusht_plan_s* p, const double* ring, void* torus, int nmaps, int f32,
                  hipStream_t s, double sgn = 1.0);
int launch_fold(const nusht_plan_s* p, const void* torus, double* ring, int nmaps, int f32,
                hipStream_t s, double sgn = 1.0);
int launch_deconv_pad(const nusht_plan_s* p, const void* tspec, void* fspec, int nmaps, int fused,
                      int f32, hipStream_t s);
int launch_deconv_trunc(const nusht_plan_s* p, const void* fspec, void* tspec, int nmaps,
                        int fused, int f32, hipStream_t s);
// band spectrum [mmax+1][n1] <-> row spectrum [n1][rw] of one map, rows [0, fine_ra) and
// [n1 - fine_rb, n1) only (rw = n2/2+1 for the rocFFT row plans, mmax+1 for the row kernels).
// band_to_rows zero-fills the columns mmax+1 .. rw-1; rows_to_band writes zeros for the rows
// no window reaches, unless window_only (the fused theta pass reads the window rows only).
int launch_band_to_rows(const nusht_plan_s* p, const void* band, void* rows, int rw,
                        hipStream_t s);
int launch_rows_to_band(const nusht_plan_s* p, const void* rows, int rw, void* band,
                        hipStream_t s, bool window_only = false);

// ---- fine-grid row transforms for n2 / 2 = 2^K or 5 2^K (rowfft.hip) ----
bool rowfft_supported(const nusht_geometry& g);
// window rows of one map: rows [n1][rw] (columns 0 .. mmax) <-> real fine grid [n1][n2]
int launch_row_c2r(const nusht_plan_s* p, const void* rows, int64_t rw, void* fine, hipStream_t s);
int launch_row_r2c(const nusht_plan_s* p, const void* fine, void* rows, int64_t rw, hipStream_t s);
// theta pass fused with the deconvolution, maps [0, nmaps): torus spectrum cs [b][mmax+1][N_t]
// <-> band spectrum [b][mmax+1][n1] (window rows only)
bool thetafft_supported(const nusht_geometry& g);
int launch_theta_inv(const nusht_plan_s* p, const void* cs, void* band, int nmaps, hipStream_t s);
int launch_theta_fwd(const nusht_plan_s* p, const void* band, void* cs, int nmaps, hipStream_t s);

// ---- nonuniform part (nufft_*.hip) ----
int launch_interp(const nusht_plan_s* p, const void* fine, double* out, int nmaps, int f32,
                  hipStream_t s);
int launch_interp_deriv(const nusht_plan_s* p, const double* fine, double* out, double* dth,
                        double* dph, int nmaps, hipStream_t s);

// ---- point binning (plan.hip) ----
int bin_points(nusht_plan_s* p, const double* theta, const double* phi, hipStream_t s);

}  // namespace nusht

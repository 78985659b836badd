// Host-side entry points of the kernels (implemented in kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

namespace xs21 {

// Element types; values match xs21_dtype.
constexpr int kF32 = 0;
constexpr int kF64 = 1;
constexpr int kBF16 = 2;

int axis_tile(int n);                   // inner columns per block of the strided passes
long axis_tiles(int n, long inner);     // blocks along the inner dimension
long bins_tiles(int n);                 // column tiles per spectrum of the binning z pass
// partial sums per spectrum written by the binning pass (<= live tiles) for a
// launch of about `blocks` blocks over `outer` spectra (blocks <= 0: default)
long bins_parts(int n, long outer, long blocks = 0);
int ion_grid(int n, int blocks = 0);    // blocks of the ionisation pass (blocks <= 0: default)
int ion_grid_max(int n);                // the largest grid ion_grid may return
int max_group();                        // walkers per ionisation launch
int max_radii();                        // radii per ladder
int thr_stride();                       // padded thresholds per walker (+inf beyond use)
int max_bins();                         // bins per spectrum
int half_pitch(int n);                  // row pitch (complex values) of a half spectrum

// Real rows [nrows][n] of `dtype` -> half-spectrum rows [nrows][half_pitch(n)].
// With nyq != nullptr (one n^3 field, nrows = n^2) the kx = n/2 entries go to
// the Nyquist plane nyq[y][z] instead of the rows.
hipError_t launch_rows_r2c(int dtype, int n, const void* in, void* out, void* nyq, long nrows, const void* tw,
                           int ntab, hipStream_t s);
// Half-spectrum rows -> real rows * scale, stored as `storage`, for `batch`
// radii: radius b reads in + b * istride and writes out + b * ostride
// (elements); entries with kx > cut[2 b + 1] (its kmax) are taken as zero
// without being read.
hipError_t launch_rows_c2r(int dtype, int storage, int n, const void* in, void* out, long nrows, double scale,
                           const long* cut, int batch, long istride, long ostride, const void* tw, int ntab,
                           hipStream_t s, int blocks = 0);
// Transform along the middle axis of [outer][n][inner] for columns < ilim
// (dir -1 forward, +1 inverse), for `batch` slices: slice b reads src + b *
// sstride and writes dst + b * dstride (elements).  mode 0 plain; mode 1 the
// z pass of a sharp-k smoothing with cutoff |n|^2 <= cut[2 b] (columns
// outside the disk skipped); mode 2 the y pass of a smoothing (only entries
// with ny^2 + kx^2 <= cut[2 b] read, columns kx <= cut[2 b + 1]); mode 4 an
// inverse z pass weighting each mode by nz^2 / |n|^2 (the line-of-sight
// velocity gradient).  cut is a device array of (n2max, kmax) pairs, used by
// modes 1 and 2 only.
hipError_t launch_axis(int dtype, int n, int dir, int mode, const void* src, void* dst, long outer, long inner,
                       long ilim, const long* cut, int batch, long sstride, long dstride, const void* tw, int ntab,
                       hipStream_t s);
// Columns per tile of the strided passes at size n (tile t covers flat
// columns t * cols .. t * cols + cols - 1 of a padded half spectrum).
int axis_tile_cols(int n);
// Columns per tile of the binning pass at size n (its live-tile lists use it).
int bins_tile_cols(int n);
// Mode 1 of launch_axis over a list of live tiles only: ntiles entries
// tiles[k] = (r << 24) | tile, each a tile with at least one column inside
// the disk |n|^2 <= cut[2 (r - r0)] of radius r of the batch starting at r0;
// radius r - r0 writes dst + (r - r0) * dstride.  src, inner and cut as in
// mode 1 (one source spectrum for every radius).
hipError_t launch_axis_live(int dtype, int n, const void* src, void* dst, long inner, const int32_t* tiles,
                            long ntiles, int r0, const long* cut, long dstride, const void* tw, int ntab,
                            hipStream_t s);
// Mode 2 of launch_axis (in place, slices [n][n][inner] at data + (r - r0) *
// stride) over a list of live column tiles: tiles[k] = (r << 24) | tile with
// tile * cols <= cut[2 (r - r0) + 1] (kmax of radius r); every z slice of
// each listed tile is transformed.  ilim: the batch's largest kmax + 1.
hipError_t launch_axis_live_y(int dtype, int n, void* data, long inner, long ilim, const int32_t* tiles, long ntiles,
                              int r0, const long* cut, long stride, const void* tw, int ntab, hipStream_t s);
// Forward z pass of `outer` padded spectra [n][n][half_pitch(n)] (kx < n/2)
// and their Nyquist planes nyq[outer][ky][z], fused with |X|^2 binning into
// part[outer][parts][nbins] (FP64); parts in [1, bins_tiles(n)], normally
// bins_parts(n, outer).  bintab / bintab_host: the bin of every |n|^2 on the
// device and on the host (the host copy sizes each launch's FP64 slots).
// The tiles are entries [0, ntiles) of the device list `tiles` (normally
// bins_live_tiles(n): no other tile holds a binned mode).
hipError_t launch_axis_bins(int dtype, int n, const void* src, const void* nyq, long outer, long parts,
                            const int32_t* tiles, long ntiles, const int8_t* bintab, const int8_t* bintab_host,
                            int nbins, double* part, const void* tw, int ntab, hipStream_t s);
// Tiles of the binning pass holding a column with ny^2 + kx^2 <= (n/2)^2.
std::vector<int32_t> bins_live_tiles(int n);
long bins_live_count(int n);
// Forward y pass, in place, of `outer` slices [n][inner] over columns
// [0, ilim) of spectra that are only binned afterwards: outputs with
// ny^2 + kx^2 > (n/2)^2 are not stored (kx = the column index, or n/2 for
// every column when nyquist, the Nyquist plane [ky][z]).
hipError_t launch_axis_fwd_disk(int dtype, int n, void* data, long outer, long inner, long ilim, bool nyquist,
                                const void* tw, int ntab, hipStream_t s, int blocks = 0);
// Ionisation + dT_b + forward x pass for nw walkers on one box: spectra
// [nw][n][n][half_pitch(n)] with kx < n/2, Nyquist planes nyq[nw][y][z].
// zt == nullptr: constant efficiency, thr[w][max_radii()]; else the
// two-population efficiency, thr[w][2][max_radii()] (lo, hi) and the cell
// radius tables zt[w][kZetaPitch] written by launch_plan2.
// field_walker >= 0: walker field_walker of the group also writes its x_HI
// and dT_b boxes (n^3 values of dtype each) to x_hi and dtb, from the same
// launch (field_walker < 0: no fields, x_hi / dtb ignored).
// slot_tab: device scratch of slot_table_bytes() for the sorted flag test of
// FP32 constant-efficiency walkers (nullptr: one compare per walker and radius).
// blocks: grid of the pass (<= 0: ion_grid's default; at most ion_grid_max);
// flag_test: 1 sorted tables, 0 one compare per walker and radius, -1 default
// (sorted unless XS21_ION_FLAGS=ballot).  The x_HI partial sums xpart hold
// one value per walker and block of the grid used.
size_t slot_table_bytes();
hipError_t launch_ion(int dtype, int storage, int n, const void* dR, const void* odens, int nr, const void* wc,
                      const void* thr, const void* zt, int nw, double tb, double dc, void* spec, void* nyq,
                      double* xpart, const void* tw, int ntab, hipStream_t s, int field_walker = -1,
                      void* x_hi = nullptr, void* dtb = nullptr, void* slot_tab = nullptr, int blocks = 0,
                      int flag_test = -1);
// Two-population planning (Section 4, eq. 9) of nw walkers on one box:
// slots[nr] (device, slot 0 = cell radius), wp[nw] (device) -> thresholds
// thr[w][2][stride] (lo, hi; +inf where unused), wc[w].upper set where some
// hi is finite (wc[w].upper must be 0 before), and the cell-radius
// effective-efficiency tables zt[w][pitch], in `dtype`.
struct SlotPlan2;
struct WalkerPlan2;
hipError_t launch_plan2(int dtype, const SlotPlan2* slots, int nr, const WalkerPlan2* wp, int nw, void* wc,
                        void* thr, int stride, void* zt, int pitch, double dc, hipStream_t s);
// Planning from device walker parameters (the sampler): constant-efficiency
// rows par[nw][3] -> walker constants wc[nw] and thresholds thr[nw][stride];
// two-population rows par[nw][5] -> wc[nw] and the inputs wp[nw] of launch_plan2.
struct BoxPlan;
struct SamplerSpec;
hipError_t launch_plan1(int dtype, const double* par, int nw, const BoxPlan& b, const SlotPlan2* slots, void* wc,
                        void* thr, int stride, hipStream_t s);
hipError_t launch_walker2(int dtype, const double* par, int nw, const BoxPlan& b, const SlotPlan2* slots, void* wc,
                          WalkerPlan2* wp, hipStream_t s);
// Stretch-move proposals of walkers k0 .. k0 + count - 1 (partners among the
// `half` walkers from o0), their acceptance given chi^2, and ln p of walkers.
hipError_t launch_propose(const double* x, int k0, int o0, int half, int count, const double* u,
                          const SamplerSpec& spec, double* prop, double* aux, hipStream_t s);
hipError_t launch_accept(double* x, double* lp, int k0, int count, int d, const double* u, const double* prop,
                         const double* aux, const double* chi2, int32_t* accepted, hipStream_t s);
hipError_t launch_lnprob(const double* x, int count, const SamplerSpec& spec, const double* chi2, double* lp,
                         hipStream_t s);
// Deterministic reduction of the bin and x_HI partial sums, one walker per block.
hipError_t launch_finalize(int nwalkers, const double* part, long ntiles, int nbins, const double* xpart, long nblk,
                           const double* counts, double pscale, double inv_cells, double* pk, long pk_stride,
                           int nbins_out, double* xhi, long xhi_stride, hipStream_t s);
// chi^2 of one box for nw walkers from their P(k) rows pk + w * pk_stride:
// tab = [k_b^3 / (2 pi^2)][mock Delta^2][variance, 0 = bin not fitted], each
// nbins long; adds to chi2[w], or sets it when first != 0.
hipError_t launch_chi2(const double* pk, long pk_stride, int nw, const double* tab, int nbins, double* chi2,
                       int first, hipStream_t s);
// odens = (1 + delta) / (1 + clamp(-g, -tmax, tmax)) per cell (g == nullptr:
// 1 + delta), the density factor of dT_b with the velocity-gradient term.
hipError_t launch_los_factor(int dtype, const void* delta, const void* g, void* odens, size_t count, double tmax,
                             hipStream_t s);
// Bandwidth probe `kind` (0 read, 1 write, 2 copy first half -> second half,
// 3 strided 128-byte tiles of 256^3 half spectra) over buf[0, bytes); sink:
// probe_sink_bytes() of device memory for the read kernels' block sums;
// *moved: HBM bytes one launch reads plus writes.
size_t probe_sink_bytes();
size_t probe_tile_spectrum_bytes();
hipError_t launch_probe(int kind, void* buf, size_t bytes, float* sink, double* moved, hipStream_t s);
// y[i] = erfc(x[i]) for `count` values by the FP32 erfc of the ionisation pass.
hipError_t launch_erfc(const float* x, float* y, size_t count, hipStream_t s);
// out[i] = (dtype) in[i] for `count` stored values.
hipError_t launch_cast(int dtype, int storage, const void* in, void* out, size_t count, hipStream_t s);

}  // namespace xs21

/*
 * fpcf4.h -- C ABI of libfpcf4, an MI355X (gfx950) implementation of the
 * multipole-based estimator of the shear four-point correlation function
 * (Porth, Silvestre-Rosello, Schneider & Larma 2025, arXiv:2509.07974).
 *
 * Problem statement (Sect. 3): N galaxies at flat-sky positions theta_i with
 * Cartesian complex shears gamma_c,i = g1 + i g2 and weights w_i; radial bins
 * Theta_b; a largest multipole nmax.  The result is the multipole tensor
 *
 *   Upsilon_{mu,(n2,n3)}(T1,T2,T3),  mu = 0..7 (x-projection, Sect. 2.2),
 *   N_{(n2,n3)}(T1,T2,T3)            (the normalisation, Sect. 3.1),
 *
 * for |n2|,|n3| <= nmax, summed over all quadruplets of *distinct* galaxies
 * (double- and triple-counting corrections of Appendix A.1 subtracted), or
 * over all index quadruplets when subtract_degenerate == 0.
 *
 * Conventions shared by every call:
 *  - All calls return fpcf4_status (0 = OK, < 0 = error).  No C++ exception
 *    crosses the ABI.  On error, fpcf4_last_error() returns a message for the
 *    calling thread.  Invalid arguments are detected before any device work.
 *  - The caller owns every input and output buffer.  The library owns only
 *    the device workspace it allocates inside a call (freed before return),
 *    except in the request API where the caller passes the workspace.
 *  - Radial bin b is the half-open interval [edges[b], edges[b+1]), decided
 *    on r^2 = dx*dx + dy*dy (two products and one sum in IEEE binary64, no
 *    fused multiply-add) against the squared edges edges[b]*edges[b]
 *    (Sect. 2.3 and 3: the bin selection function).  Pairs closer than
 *    edges[0] or at least edges[nbins] apart are not counted.
 *  - Position angles phi_ij = atan2(y_j - y_i, x_j - x_i), counter-clockwise
 *    from +x (Sect. 2.2).  No periodic wrap.
 *  - Device pointers are HIP device pointers on the current device; `stream`
 *    is a hipStream_t on which every device operation of the call is
 *    queued (NULL = the HIP null stream).  The library does not order that
 *    stream after work the caller queued on other streams: inputs written on
 *    another stream must be complete (or the stream made to wait) before the
 *    call.  The estimate calls are synchronous: results are complete in the
 *    output buffer on return.
 */
#ifndef FPCF4_H
#define FPCF4_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t fpcf4_status;

enum {
  FPCF4_OK = 0,
  FPCF4_E_INVALID_ARG = -1,   /* bad pointer, size, edge array, non-finite input */
  FPCF4_E_UNSUPPORTED = -2,   /* nmax or nbins beyond the compiled limits        */
  FPCF4_E_OUT_OF_MEMORY = -3, /* device allocation failed                         */
  FPCF4_E_DEVICE = -4,        /* a HIP runtime call or kernel launch failed       */
  FPCF4_E_BUDGET = -5,        /* caller workspace smaller than fpcf4_plan() says  */
  FPCF4_E_CANCELLED = -6      /* request cancelled                                */
};

enum { FPCF4_MEM_HOST = 0, FPCF4_MEM_DEVICE = 1 };

/* Arithmetic of the path.
 *  FPCF4_FP64       : every stage in binary64.
 *  FPCF4_MIXED_FP16 : pair multipoles accumulated in binary32 with blocked
 *                     summation into binary64; contraction on MFMA with
 *                     fp16 hi/lo split operands and fp32 accumulation per
 *                     centre chunk; binary64 cross-chunk reduction,
 *                     degenerate-term subtraction and output.
 *  FPCF4_MIXED_BF16 : as FP16 with bf16 hi/lo split operands. */
enum { FPCF4_FP64 = 0, FPCF4_MIXED_FP16 = 1, FPCF4_MIXED_BF16 = 2 };

#define FPCF4_NMAX_SUPPORTED 16   /* largest nmax compiled in              */
#define FPCF4_NBINS_SUPPORTED 128 /* largest number of radial bins         */
#define FPCF4_NMAX3_SUPPORTED 32  /* largest 3PCF multipole (2 x the above) */
#define FPCF4_NCORR 9             /* Upsilon_0..7 and N                    */

/* Catalogue: structure of arrays of length n, caller-owned, read-only.
 * Positions in any flat-sky unit (the edges use the same unit).  All values
 * must be finite; weights may have any sign. */
typedef struct {
  int64_t n;
  const double *x, *y;    /* positions                                     */
  const double *g1, *g2;  /* gamma_c = g1 + i g2, in the same x/y frame     */
  const double *w;        /* weights                                       */
  int32_t mem;            /* FPCF4_MEM_HOST or FPCF4_MEM_DEVICE             */
} fpcf4_catalogue;

/* Radial bins: nbins + 1 strictly increasing finite edges, edges[0] > 0.
 * Host memory. */
typedef struct {
  int32_t nbins;
  const double *edges;
} fpcf4_bins;

typedef struct {
  int32_t nmax;                /* 0 <= nmax <= FPCF4_NMAX_SUPPORTED          */
  int32_t precision;           /* FPCF4_FP64 / FPCF4_MIXED_FP16 / _BF16       */
  int32_t subtract_degenerate; /* 1 = distinct quadruplets, 0 = raw sums      */
  int32_t reserved;
  const int64_t *centers;      /* optional: indices of the galaxies used as
                                  base point X_0 (in catalogue memory space);
                                  NULL = all.  Every galaxy stays a neighbour. */
  int64_t ncenters;
  int64_t tile_centers;        /* centres per stage tile; 0 = planner choice  */
  void *stream;                /* hipStream_t, or NULL for the null stream    */
} fpcf4_options;

/* Number of complex128 elements of the output tensor:
 * 9 * nbins^3 * (2 nmax + 1)^2. */
int64_t fpcf4_output_elems(int32_t nbins, int32_t nmax);

/* Full estimate (Sect. 3.1 multipoles, App. A.1 corrections).
 * upsilon: caller-owned complex128 array, interleaved (re, im), layout
 *   [9][nbins][nbins][nbins][2nmax+1][2nmax+1], index 0..7 = Upsilon_mu,
 *   8 = N; the multipole n2 (n3) is stored at offset n2 + nmax (n3 + nmax).
 * out_mem: FPCF4_MEM_HOST or FPCF4_MEM_DEVICE for `upsilon`.
 * N < 1 or no pair in range gives zeros with FPCF4_OK. */
fpcf4_status estimate_4pcf_multipoles(const fpcf4_catalogue *cat,
                                      const fpcf4_bins *bins,
                                      const fpcf4_options *opts,
                                      double *upsilon, int32_t out_mem);

/* Bytes of the static device scratch of estimate_4pcf_multipoles_noalloc. */
#define FPCF4_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* estimate_4pcf_multipoles for callers that cannot allocate device memory
 * (serving loops that must not call hipMalloc, harnesses that forbid it):
 * same arguments, output and errors, but the workspace is a static device
 * array of FPCF4_NOALLOC_SCRATCH_BYTES (64 MiB) that each GPU the library
 * runs on holds until the process ends; no device memory is allocated or
 * freed.  With opts->tile_centers == 0 the centre tile is halved until the
 * workspace fits; a workspace that still does not fit (or does not fit at
 * the caller's tile) fails with FPCF4_E_BUDGET before any device work.
 * Every call on one GPU uses the same array, and each call re-initialises
 * what must start at zero: calls are serialised within this process, and
 * calls from other processes on the same GPU race and must not overlap.
 * The call waits for `stream` before returning. */
fpcf4_status estimate_4pcf_multipoles_noalloc(const fpcf4_catalogue *cat,
                                              const fpcf4_bins *bins,
                                              const fpcf4_options *opts,
                                              double *upsilon, int32_t out_mem);

/* Number of complex128 elements of the 3PCF output: 5 * nbins^2 * (2 nmax + 1). */
int64_t fpcf4_output3_elems(int32_t nbins, int32_t nmax);

/* Shear 3PCF multipoles through the order-N construction of the appendix on
 * N-th order shear statistics, at N = 3 (natural components Gamma_0..Gamma_3
 * from the beta matrix, generalised x-projection zeta_0 = (phi_1 + phi_2)/2):
 *   Upsilon_{mu,n}(T1, T2) = s_mu sum_i x_i F1 F2 with
 *   mu 0: x = w g,  F1 = G_{n-3},         F2 = G_{-n-3};
 *   mu 1: x = conj(w g), F1 = G_{n-1},    F2 = G_{-n-1};
 *   mu 2: x = w g,  F1 = conj G_{-n-1},   F2 = G_{-n-3};
 *   mu 3: x = w g,  F1 = G_{n-3},         F2 = conj G_{n-1};
 *   N   : x = w,    F1 = W_n,             F2 = W_{-n}
 * with s_mu = -1 for mu = 0..3 and +1 for N: the natural components are
 * products of three projected shears gamma = -gamma_c e^{-2i zeta} (Sect.
 * 2.1), whose factor (-1)^3 the block formula of that appendix leaves out.
 * The blocks come from the stage (a) records of order ceil(nmax / 2), so the
 * pair stage is shared with the 4PCF path.
 * opts->nmax is the largest 3PCF multipole, 0 <= nmax <= FPCF4_NMAX3_SUPPORTED;
 * opts->precision selects the stage (a) accumulation (the contraction is
 * binary64 in every mode); subtract_degenerate = 1 removes the terms with
 * the same neighbour in both slots (distinct triplets).
 * upsilon3: caller-owned complex128 (re, im) array
 *   [5][nbins][nbins][2nmax+1], index 0..3 = Upsilon_mu, 4 = N, n stored at
 *   offset n + nmax; host or device memory as out_mem says.
 * Errors as for estimate_4pcf_multipoles; FPCF4_E_UNSUPPORTED for nmax > 32. */
fpcf4_status estimate_3pcf_multipoles(const fpcf4_catalogue *cat,
                                      const fpcf4_bins *bins,
                                      const fpcf4_options *opts,
                                      double *upsilon3, int32_t out_mem);

/* Tree approximation of the per-centre multipoles (Sect. 3, practical
 * implementation): a hierarchy of grids of cell side delta1 * 2^(d-1),
 * d = 1..nlevels; every non-empty cell becomes one pseudo-galaxy at its
 * w-weighted centre of mass carrying the cell sums of w gamma, w and of the
 * multiple-counting weights; a radial bin takes its neighbours from the
 * coarsest grid with edges[b] / Delta_d >= rmin, or from the galaxies when
 * none qualifies.  Centres remain the galaxies.  Grids are anchored at the
 * catalogue's minimum x and y. */
typedef struct {
  int32_t nlevels;             /* 1 .. 4                                      */
  int32_t reserved;
  double delta1;               /* finest cell side (arcmin), > 0              */
  double rmin;                 /* >= 2                                        */
} fpcf4_tree;

/* estimate_4pcf_multipoles with the tree approximation (same output).
 * Mixed precisions only (FPCF4_E_UNSUPPORTED for FPCF4_FP64); invalid tree
 * parameters give FPCF4_E_INVALID_ARG.  With no bin qualifying for a grid
 * the result equals estimate_4pcf_multipoles. */
fpcf4_status estimate_4pcf_multipoles_tree(const fpcf4_catalogue *cat,
                                           const fpcf4_bins *bins,
                                           const fpcf4_options *opts,
                                           const fpcf4_tree *tree,
                                           double *upsilon, int32_t out_mem);

/* Shear 3PCF multipoles (as estimate_3pcf_multipoles) with the BaseTree and
 * Tree approximations of the appendix on N-th order statistics (its
 * subsection on the algorithmic implementation); both together are the
 * DoubleTree approximation.
 * base (may be NULL): the base points X_0 are the pseudo-galaxies of a
 *   hierarchy of grids of cell side base->delta1 * 2^(d-1), d = 1 ..
 *   base->nlevels (anchored, centred and summed as for the tree
 *   approximation, fpcf4_tree below), each carrying the cell sums of w gamma
 *   and w as its centre value; radial bin b uses the coarsest grid with
 *   edges[b] / Delta_d >= base->rmin, or the galaxies when none qualifies.
 *   For a bin pair the centre value times the block of the bin on the finer
 *   grid is summed over the cells of that grid inside each cell of the
 *   coarser grid (cells are nested) and multiplied there by the other bin's
 *   block.  Every galaxy is a base point (FPCF4_E_INVALID_ARG for
 *   opts->centers) and the records of all galaxies must fit one centre tile
 *   (FPCF4_E_UNSUPPORTED otherwise).
 * tree (may be NULL): the blocks of radial bin b are allocated over the
 *   pseudo-galaxies of the coarsest neighbour grid with
 *   edges[b] / Delta_d >= tree->rmin (as in estimate_4pcf_multipoles_tree),
 *   with the cell sums of the product weights in the same-neighbour terms.
 * The same-neighbour terms are removed where Theta_1 = Theta_2.  With no bin
 * reaching a grid of either hierarchy the result equals
 * estimate_3pcf_multipoles.  Mixed precisions only when base or tree is
 * given (FPCF4_E_UNSUPPORTED for FPCF4_FP64).  Output and other errors as
 * estimate_3pcf_multipoles. */
fpcf4_status estimate_3pcf_multipoles_doubletree(const fpcf4_catalogue *cat,
                                                 const fpcf4_bins *bins,
                                                 const fpcf4_options *opts,
                                                 const fpcf4_tree *base,
                                                 const fpcf4_tree *tree,
                                                 double *upsilon3, int32_t out_mem);

/* Stage (a) only, for parity checks (Sect. 3.1: the per-centre blocks G_n and
 * W_n "defined as in P24", read as G_k = sum_j w_j gamma_j e^{+ik phi_ij} and
 * W_k = sum_j w_j e^{+ik phi_ij} over neighbours j in the bin).
 * For the centres of opts (or all), in that order, writes
 *   counts[c][b]  : number of neighbours in bin b (int64, may be NULL),
 *   G[c][b][k]    : complex128 (re, im), k = -2nmax-3 .. 2nmax-1 (may be NULL),
 *   W[c][b][k]    : complex128, k = -2nmax .. 2nmax (may be NULL).
 * All outputs in host memory.  Uses opts->precision for the accumulation.
 * Without opts->centers every galaxy is reported, in catalogue order; a
 * device-memory catalogue then needs an explicit centre list. */
fpcf4_status fpcf4_debug_multipoles(const fpcf4_catalogue *cat,
                                    const fpcf4_bins *bins,
                                    const fpcf4_options *opts,
                                    int64_t *counts, double *G, double *W);

/* The contraction plan of stage (b), for checks (host only: no device work).
 * Every Upsilon_{mu,(n2,n3)} (Sect. 3.1) is a sum over centres of x times
 * one block at each of Theta_1, Theta_2, Theta_3; the plan forms each
 * distinct product of three blocks once, as a row block times a pair of
 * column blocks, and reads the other (mu, n2, n3) with the same blocks at
 * permuted bins (the radial symmetry of Table 2).  For every (mu, n2, n3),
 * in the order of the output tensor, writes 16 int32 to out (host memory,
 * 9 (2nmax+1)^2 * 16 values):
 *   [0]      centre factor: 0 = w gamma, 1 = its conjugate, 2 = w
 *   [1..3]   row block: family (0 = G, 1 = W), conjugated (0/1), order k
 *   [4..6]   first column block: family, conjugated, order
 *   [7..9]   second column block: family, conjugated, order
 *   [10..12] which of (b1, b2, b3) (0, 1, 2) gives the bin of the row block,
 *            of the first and of the second column block
 *   [13]     work item, [14] row block within it, [15] row blocks of the item
 * *nitems (may be NULL) receives the number of work items.
 * FPCF4_E_INVALID_ARG for nmax outside [0, FPCF4_NMAX_SUPPORTED] or a null out. */
fpcf4_status fpcf4_debug_pair_plan(int32_t nmax, int32_t *out, int64_t *nitems);

/* The degenerate-term sums of the subtraction (App. A.1, Table 1), for checks
 * (host only: no device work).  Every entry of the correction buffer is
 * sum_i x_i E_i(b) F_i(b'): E the Table 1 block at the equal bins, F the
 * remaining factor at the other bin (F = 1 for the triple term); the
 * library forms each distinct (x, E, F) once.  For every mu and slot (the
 * 2nmax+1 orders n3 of Theta_1 = Theta_2, the 2nmax+1 orders n2 of
 * Theta_1 = Theta_3, the 4nmax+1 orders n2 + n3 of Theta_2 = Theta_3, then
 * the triple term), writes 8 int32 to out (host memory,
 * 9 (8 nmax + 4) * 8 values):
 *   [0] centre factor: 0 = w gamma, 1 = its conjugate, 2 = w
 *   [1] E family: 2 = Q, 3 = A, 4 = V, 5 = T, 6 = M, 7 = U;  [2] E order
 *   [3] F family: 0 = G, 1 = W, -1 for the triple term; [4] F conjugated;
 *   [5] F order;  [6] the distinct sum;  [7] 0
 * *nsums (may be NULL) receives the number of distinct sums.
 * FPCF4_E_INVALID_ARG for nmax outside [0, FPCF4_NMAX_SUPPORTED] or a null out. */
fpcf4_status fpcf4_debug_corr_plan(int32_t nmax, int32_t *out, int64_t *nsums);

/* The stable radix sort of the cell-list build, for checks (the spatial sort
 * that puts the neighbours of the pair sums of Sect. 3.1 / App. A cell by
 * cell, and the cells of the reduced catalogues of Sect. 3.2).  Sorts the n
 * (key, value) pairs by key, equal keys keeping their input order, on the
 * device (key_bytes 4: 32-bit keys, as the cell and Morton keys; 8: 64-bit,
 * as the reduced-catalogue cells).  keys, vals (inputs) and keys_out,
 * vals_out (outputs) are host arrays of n entries; keys are passed as
 * uint64 in both cases.  FPCF4_E_INVALID_ARG for n outside [0, 2^31),
 * key_bytes not 4 or 8, key_bits outside [1, 8 key_bytes], a key not below
 * 2^key_bits or a null array with n > 0; FPCF4_E_DEVICE on a device error. */
fpcf4_status fpcf4_debug_sort_pairs(const uint64_t *keys, const int32_t *vals, int64_t n,
                                    int32_t key_bits, int32_t key_bytes, uint64_t *keys_out,
                                    int32_t *vals_out);

/* Conversion to bin-averaged natural components (Sect. 2.3 and Eq. of the
 * multipole expansion in Sect. 3.1): for nphi linear angular bins on
 * [0, 2pi),
 *   Ubar_mu(T, Phi_a, Phi_b) = (2pi)^-2 sum_n Upsilon_mu,n I_n2(Phi_a) I_n3(Phi_b),
 *   I_0 = |Delta Phi|, I_m = (e^{i m Phi_up} - e^{i m Phi_low}) / (i m),
 * and Gamma_mu = Ubar_mu / Nbar (0 where Nbar == 0).
 * upsilon: host complex128 [9][nb][nb][nb][2nmax+1][2nmax+1] (as produced
 * above); gamma_out: host complex128 [8][nb][nb][nb][nphi][nphi];
 * norm_out: host double [nb][nb][nb][nphi][nphi] (Re Nbar), may be NULL.
 * Computed in binary64 on the device. */
fpcf4_status fpcf4_to_natural(const double *upsilon, int32_t nbins,
                              int32_t nmax, int32_t nphi, double *gamma_out,
                              double *norm_out, void *stream);

/* The same conversion for a caller-chosen list of radial-bin triplets only,
 * so that a large multipole tensor can be turned into natural components
 * block by block without materialising nbins^3 * nphi^2 values (device
 * memory used: about 9 * ntrip * ((2nmax+1)^2 + nphi (2nmax+1) + nphi^2)
 * complex128 plus the input when it is on the host).
 * upsilon: [9][nbins][nbins][nbins][2nmax+1][2nmax+1] complex128 as returned
 *   by estimate_4pcf_multipoles, in host or device memory (ups_mem).
 * triplets: host int32 [ntrip][3] = (b1, b2, b3), each in [0, nbins).
 * gamma_out: complex128 [8][ntrip][nphi][nphi]; norm_out (may be NULL):
 *   float64 [ntrip][nphi][nphi]; both in host or device memory (out_mem).
 * Same angular binning, normalisation and zero rule as fpcf4_to_natural;
 * synchronous with respect to `stream` on return.  0 <= ntrip <= 2^24. */
fpcf4_status fpcf4_to_natural_triplets(const double *upsilon, int32_t ups_mem,
                                       int32_t nbins, int32_t nmax, int32_t nphi,
                                       const int32_t *triplets, int64_t ntrip,
                                       double *gamma_out, double *norm_out,
                                       int32_t out_mem, void *stream);

/* ------------------------------------------------------------------------
 * Request API for serving: the caller sizes and owns the device workspace
 * (admission by HBM footprint), then advances the request one centre tile
 * at a time on the request's stream.  A request never allocates.
 * ---------------------------------------------------------------------- */
typedef struct fpcf4_request fpcf4_request;

/* Device bytes of workspace and number of centre tiles that a request with
 * these inputs needs.  Catalogue pointers are not read (may be NULL); only
 * cat->n, the bins and the options matter. */
fpcf4_status fpcf4_plan(const fpcf4_catalogue *cat, const fpcf4_bins *bins,
                        const fpcf4_options *opts, size_t *device_bytes,
                        int64_t *ntiles);

/* Bind inputs and a caller workspace (device memory of at least the planned
 * size, 256-byte aligned).  Uploads the catalogue and builds the cell list
 * on opts->stream.  The catalogue may be freed once this returns. */
fpcf4_status fpcf4_request_create(const fpcf4_catalogue *cat,
                                  const fpcf4_bins *bins,
                                  const fpcf4_options *opts,
                                  void *device_workspace, size_t bytes,
                                  fpcf4_request **req);

/* Enqueue stage (a), stage (b) and the correction sums of one centre tile
 * (0 <= tile < ntiles, each tile exactly once, any order) on the request's
 * stream.  Returns without waiting for the GPU. */
fpcf4_status fpcf4_request_step(fpcf4_request *req, int64_t tile);

/* Apply the degenerate-term subtraction and copy the result (layout as for
 * estimate_4pcf_multipoles) into `upsilon`; waits for the request's stream.
 * Fails with FPCF4_E_INVALID_ARG unless every tile has been stepped. */
fpcf4_status fpcf4_request_finalize(fpcf4_request *req, double *upsilon,
                                    int32_t out_mem);

/* Release the request handle (not the caller's workspace). NULL is a no-op. */
void fpcf4_request_destroy(fpcf4_request *req);

/* ------------------------------------------------------------------------
 * Per-stage timing for measurement.  While enabled, every request step
 * records hipEvents on the request's stream around the stage (a) pair
 * kernel (pair multipoles), the relayout of its records to centre-contiguous
 * rows, stage (b) (contraction) and the correction sums, and counts the
 * ordered (centre, neighbour) pairs that fell in a bin; totals are
 * accumulated when a request is finalized.  Times in milliseconds.
 * ---------------------------------------------------------------------- */
typedef struct {
  double stage_a_ms;    /* pair-multipole kernel                          */
  double relayout_ms;   /* record relayout [centre][bin][entry] -> rows    */
  double stage_b_ms;    /* contraction                                   */
  double corr_ms;       /* degenerate-term sums                          */
  int64_t stage_a_launches, stage_b_launches, steps, pairs, centres;
  double stage_b_mfma_flops;  /* matrix-core flops the contraction issued
                                 (padding and hi/lo products included)    */
  double stage_b_useful_flops; /* 8 per complex multiply-add of the distinct
                                  block products it formed (every bin
                                  triple of every distinct product)       */
} fpcf4_profile;

/* Enable (on != 0) or disable timing; either call resets the totals. */
fpcf4_status fpcf4_profile_enable(int32_t on);

/* Copy the accumulated totals into *out. */
fpcf4_status fpcf4_profile_read(fpcf4_profile *out);

/* Message for the last failing call on this thread ("" if none). */
const char *fpcf4_last_error(void);

/* Library version string. */
const char *fpcf4_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FPCF4_H */

/*
 * sbr.h -- C-ABI of the MI355X SBR (shooting-and-bouncing-ray) channel library.
 *
 * Method: Wang et al., "An SBR Based Ray Tracing Channel Modeling Method for
 * THz and Massive MIMO Communications" (arXiv 2208.10006), Section II.  The
 * four calls follow its four steps (Sec. II-A): ray launching, ray tracing,
 * ray reception and ray calculation, with the THz corrections of Sec. II-B
 * and the MIMO outputs of Sec. II-C.
 *
 * Conventions (all calls):
 *   - SI units: metres, seconds, hertz, S/m.  Angles in degrees unless noted.
 *   - Every call returns an sbr_status; nothing throws across the ABI.  On a
 *     non-OK status no output is written, no handle is created, and
 *     sbr_last_error() (thread-local) describes the failure.  HIP runtime
 *     failures map to SBR_E_DEVICE with the HIP error string in the message.
 *   - Input arrays are borrowed for the duration of the call.  By default they
 *     are host pointers and are copied before the call returns; with
 *     SBR_IN_DEVICE they are device pointers on the context's device, read in
 *     stream order (they must stay valid until the context stream passes the
 *     call).
 *   - Output arrays are caller-allocated.  By default host pointers (the call
 *     synchronises the context stream before returning); with SBR_OUT_DEVICE
 *     device pointers written in stream order.
 *   - Handles are owned by the library until sbr_release().  A trace keeps
 *     its scene alive, a path set keeps its trace alive (reference counts).
 *   - Determinism: identical inputs give bitwise-identical outputs (sorted
 *     keys, fixed reduction orders, no floating-point atomics).
 *   - Threading: one context per host thread.
 */
#ifndef SBR_H_
#define SBR_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SBR_OK = 0,
  SBR_E_INVALID_ARG = -1,   /* bad size, NaN/Inf, degenerate triangle, ...   */
  SBR_E_OUT_OF_MEMORY = -2, /* device allocation failed                        */
  SBR_E_DEVICE = -3,        /* HIP runtime error or a kernel-reported failure  */
  SBR_E_CAPACITY = -4,      /* an output buffer is too small (size in message) */
  SBR_E_STATE = -5,         /* call order violated (e.g. stats before channel) */
  SBR_E_UNSUPPORTED = -6
} sbr_status;

#define SBR_IN_DEVICE 0x1u  /* pointer inputs are device pointers              */
#define SBR_OUT_DEVICE 0x2u /* pointer outputs are device pointers             */

#define SBR_POL_V 0 /* theta-hat of the departure / arrival direction */
#define SBR_POL_H 1 /* phi-hat of the departure / arrival direction   */

#define SBR_MAX_BOUNCES 16

typedef struct sbr_context_s* sbr_context_t; /* device, stream, tuning         */
typedef struct sbr_scene_s* sbr_scene_t;     /* triangles, face groups, BVH    */
typedef struct sbr_trace_s* sbr_trace_t;     /* per-ray hit chains ("RT tree") */
typedef struct sbr_paths_s* sbr_paths_t;     /* unique validated paths         */
typedef struct sbr_diff_s* sbr_diff_t;       /* first-order diffraction paths  */
typedef struct sbr_scat_s* sbr_scat_t;       /* first-order scattering paths   */

/* One propagation path (Sec. II-A-4: a multipath component of eq. (2)/(4)).
 * tx, rx: element indices; order: number of reflections; groups: the face
 * groups reflected from, in order (-1 padded).  Angles: AoD = direction of
 * travel leaving the Tx, AoA = direction from the Rx toward the last
 * interaction; azimuth atan2(y, x) in (-180, 180], elevation asin(z). */
typedef struct {
  int32_t tx, rx, order, flags;
  int32_t groups[SBR_MAX_BOUNCES];
  double length_m, delay_s;
  float aod_az, aod_el, aoa_az, aoa_el;
  float power; /* band mean of |a_n(f)|^2 over the last sbr_channel grid; 0 before */
  int32_t pad;
} sbr_path_record;

/* ------------------------------------------------------------------------ */
/* Context.  device: HIP ordinal.  hip_stream: a hipStream_t to run on, or
 * NULL for a library-owned stream.  Contexts are independent: calls on
 * different contexts may run at the same time from different host threads
 * (one thread per context at a time).  A handle made on one context may be
 * passed to calls on another once the work that made it has finished: scene
 * builds, batched traces and receives finish before they return; after
 * sbr_trace call sbr_synchronize on its context first.  */
sbr_status sbr_context_create(int device, void* hip_stream, sbr_context_t* out);
/* Block until all work queued by this context has finished. */
sbr_status sbr_synchronize(sbr_context_t ctx);

/* Scene (Sec. III-A: triangle scenes; Sec. II-B-1 / eq. (6)-(8): per-surface
 * relative permittivity, conductivity and roughness).
 * tri_xyz: [T][3][3] vertices (FP64, metres).  eps_r >= 1, sigma >= 0 (S/m),
 * rough_std >= 0 (m), each [T] FP32.  T = 0 is allowed (free space).
 * Triangles are double sided.  Coplanar triangles with equal materials form
 * one face group (the reflector a path key names).  Errors: INVALID_ARG on
 * NaN/Inf, negative size, bad material or a triangle of area <= 1e-12 diag^2
 * (the message names the index). */
sbr_status sbr_scene_build(sbr_context_t ctx, const double* tri_xyz, int64_t T, const float* eps_r,
                           const float* sigma_S_per_m, const float* rough_std_m, uint32_t flags,
                           sbr_scene_t* out);
/* Several scenes at once (the batched form of sbr_scene_build, for the many
 * scenes of a batched trace): scene i from tri_xyz[i] ([T[i]][3][3]) and the
 * material arrays eps_r[i], sigma_S_per_m[i], rough_std_m[i], all host or all
 * device arrays as `flags` says.  Up to 8 worker threads, each with its own
 * stream and pinned staging area, build the scenes largest first, so the host
 * work (validation, planes, face groups) of different scenes and their tree
 * builds on the GPU overlap.  The scenes are the ones sbr_scene_build would
 * return and belong to ctx like them.  Device inputs are read after the
 * context's stream has finished its earlier work.  out[i] receives scene i;
 * on error no scene is returned (out untouched) and the message names the
 * failing scene.  Not to be called concurrently on one context. */
sbr_status sbr_scene_build_batch(sbr_context_t ctx, int32_t n, const double* const* tri_xyz, const int64_t* T,
                                 const float* const* eps_r, const float* const* sigma_S_per_m,
                                 const float* const* rough_std_m, uint32_t flags, sbr_scene_t* out);

/* Launch + trace (Sec. II-A-1, II-A-2).  Every Tx element (eq. (11)) launches
 * 10 N^2 + 2 rays along the frequency-N icosahedral geodesic directions
 * (its own spherical wavefront), and each ray is reflected specularly up to
 * max_bounces times; the (max_bounces+1)-th hit absorbs it.  The per-ray hit
 * chain is kept on the device for sbr_receive.
 * tx_xyz: [Nt][3] FP64.  1 <= geodesic_N <= 46340 ("level L" = N = 2^L),
 * 0 <= max_bounces <= 16, Nt * (10 N^2 + 2) < 2^32. */
sbr_status sbr_trace(sbr_context_t ctx, sbr_scene_t scene, const double* tx_xyz, int32_t Nt,
                     int32_t geodesic_N, int32_t max_bounces, uint32_t flags, sbr_trace_t* out);
/* Batched launch + trace of n independent problems (scenes of any size, own
 * Tx arrays, launch densities and bounce limits): the rays of all of them
 * are traced by one persistent launch per bounce (breadth-first over the
 * whole batch), and out[i] is an ordinary trace handle of problem i.
 * tx_xyz[i]: [Nt[i]][3] FP64 (host pointers, or device with SBR_IN_DEVICE).
 * Sum of all rays < 2^32 - 2^22. */
sbr_status sbr_trace_batch(sbr_context_t ctx, int32_t n, const sbr_scene_t* scenes, const double* const* tx_xyz,
                           const int32_t* Nt, const int32_t* geodesic_N, const int32_t* max_bounces, uint32_t flags,
                           sbr_trace_t* out);
/* Device-side latency of a batched trace: wall-clock time (ms) from the first
 * to the last ray chunk of this problem; -1 for traces not made in a batch. */
sbr_status sbr_trace_latency(sbr_trace_t tr, double* ms);
/* rays = Nt (10N^2+2); segments = closest-hit queries actually traced. */
sbr_status sbr_trace_info(sbr_trace_t tr, int64_t* rays, int64_t* segments);
/* Per-ray hit triangles seq [rays][K+1] (original triangle index; -1 miss,
 * -2 not traced because the ray ended earlier) and, when uv is not NULL, the
 * barycentric coordinates uv [rays][K+1][2] of every hit on its triangle
 * (P = (1 - u - v) v0 + u v1 + v v2, the ray's chain replayed in FP64 on the
 * hit planes; NaN where seq < 0).  Rays by global id p R + r.  Either output
 * may be NULL, not both.  Host or device outputs (diagnostic / parity). */
sbr_status sbr_trace_hits(sbr_trace_t tr, int32_t* seq, float* uv, uint32_t flags);

/* Reception (Sec. II-A-3) and path extraction.  A segment with origin o,
 * unit direction d, end t_end and unfolded length L before it is captured by
 * Rx q when t* = (q - o).d lies in [0, t_end] and |q - o - t* d| <=
 * radius_coeff * alpha * (L + t*) / sqrt(3).  alpha_rad <= 0 selects the mean
 * great-circle angle between neighbouring geodesic rays.  Captures are
 * reduced to unique keys (Tx, Rx, face-group sequence); every key is rebuilt
 * exactly by the image method (Sec. I) in FP64 and kept only when its
 * reflection points lie on their faces, on the incidence side, unoccluded.
 * rx_xyz: [Nr][3] FP64, no Rx may coincide with a Tx. */
sbr_status sbr_receive(sbr_context_t ctx, sbr_trace_t tr, const double* rx_xyz, int32_t Nr, double alpha_rad,
                       double radius_coeff, uint32_t flags, sbr_paths_t* out);
/* capture events, distinct keys before validation, valid paths */
sbr_status sbr_paths_info(sbr_paths_t ps, int64_t* events, int64_t* keys, int64_t* paths);
sbr_status sbr_paths_count(sbr_paths_t ps, int64_t* n);
/* Capture events behind the paths (diagnostic): global ray id (tx * rays +
 * ray), receiver and segment index k of each capture, host arrays of length
 * >= events (sbr_paths_info); unordered.  Any output may be NULL. */
sbr_status sbr_paths_events(sbr_paths_t ps, int64_t capacity, uint32_t* ray, int32_t* rx, int32_t* k,
                            int64_t* written);
/* Host copy of the path list, ordered by (rx, tx, delay). */
sbr_status sbr_paths_get(sbr_paths_t ps, int64_t capacity, sbr_path_record* out, int64_t* written);

/* Ray calculation (Sec. II-A-4 and II-B): the field of every path at every
 * frequency, eq. (1) with the Kirchhoff-corrected Fresnel coefficients of
 * eq. (6)-(8), the free-space factor that eq. (3) turns into Friis for unit
 * isotropic antennas, and per-frequency specific attenuation (dB/m) and
 * dispersion (deg/m) tables standing for eq. (9)-(10) (NULL = none); then the
 * coherent sum per (f, Rx, Tx) of eq. (2) = h_qp of eq. (13)-(14):
 *   H[f][q][p] = sum over paths n of (p, q) of a_n(f).
 * a_n(f) = lambda/(4 pi d) e_rx . [prod rho R] e_tx 10^(-g d/20) e^{-j(2 pi f d/c + pi phi d/180)};
 * the phase is taken as 2 pi frac(f d / c) in FP64; the sum is FP64.
 * H_c64: [Nf][Nr][Nt] interleaved (re, im) FP32, may be NULL if H_c128 given;
 * H_c128: same shape FP64 or NULL.  Also stores each path's band-mean power. */
sbr_status sbr_channel(sbr_context_t ctx, sbr_paths_t ps, const double* freq_hz, int32_t Nf,
                       const float* atm_db_per_m, const float* atm_deg_per_m, int32_t pol_tx, int32_t pol_rx,
                       void* H_c64, double* H_c128, uint32_t flags);
/* Per-path amplitudes a_n(f), [n_paths][Nf] interleaved FP64, same arguments
 * as sbr_channel (diagnostic / parity output). */
sbr_status sbr_path_field(sbr_context_t ctx, sbr_paths_t ps, const double* freq_hz, int32_t Nf,
                          const float* atm_db_per_m, const float* atm_deg_per_m, int32_t pol_tx, int32_t pol_rx,
                          double* a_c128, uint32_t flags);

/* ------------------------------------------------------------------------ */
/* First-order edge diffraction (Sec. II-A-2 and Fig. B(b) name it, Table I
 * uses it; the paper gives no coefficient).  The uniform theory of
 * diffraction of Kouyoumjian and Pathak for straight wedges, the two
 * reflection-type terms weighted by the faces' Fresnel coefficients (TE for
 * the soft, TM for the hard coefficient) and roughness factors at the true
 * incidence angle on each face (Luebbers' form for lossy wedges).
 * Wedges: triangle edges shared by exactly two triangles of different face
 * groups whose planes are not parallel; the solid fills the smaller sector
 * between the faces (exterior angle n pi, 1 < n < 2); face 0 is the triangle
 * of lower index; wedges are numbered by (lower triangle, its edge from
 * vertex i to vertex i+1).  A path Tx -> Q -> Rx exists when Tx and Rx lie
 * strictly inside the exterior sector, Q (on Keller's cone) lies strictly
 * inside the edge, and neither leg crosses a triangle outside the wedge's two
 * face groups (the image-method margins).  Only diffraction alone is
 * modelled (no reflection before or after it).
 * sbr_diffract: tx_xyz [Nt][3], rx_xyz [Nr][3] FP64 (host, or device with
 * SBR_IN_DEVICE); finishes before it returns; the handle keeps the scene.
 * Errors: INVALID_ARG (NULL, sizes, non-finite points), UNSUPPORTED when
 * wedges x Nt x Nr >= 2^32 or 2^31 paths or more are found. */
sbr_status sbr_diffract(sbr_context_t ctx, sbr_scene_t sc, const double* tx_xyz, int32_t Nt, const double* rx_xyz,
                        int32_t Nr, uint32_t flags, sbr_diff_t* out);
/* counts: wedges of the scene, (wedge, Tx, Rx) candidates, candidates past the
 * sector and edge tests, paths (any output may be NULL) */
sbr_status sbr_diff_info(sbr_diff_t d, int64_t* wedges, int64_t* candidates, int64_t* geometric, int64_t* paths);
/* the first min(capacity, paths) paths, ordered by (Rx, Tx, wedge), to host
 * arrays: ids [n][3] int32 (tx, rx, wedge); rec [n][8] FP64 (Q xyz, s' = |Q - Tx|,
 * s = |Rx - Q|, beta0, phi', phi in radians) */
sbr_status sbr_diff_paths(sbr_diff_t d, int64_t capacity, int32_t* ids, double* rec, int64_t* written);
/* the scene's wedges in their numbering, to host arrays: geo [n][8] FP64 (start
 * xyz, end xyz, exterior angle / pi, length), groups [n][2] (face 0, face n);
 * count = number of wedges (either output may be NULL) */
sbr_status sbr_scene_wedges(sbr_context_t ctx, sbr_scene_t sc, int64_t capacity, double* geo, int32_t* groups,
                            int64_t* count);
/* H[f][q][p] += the diffracted fields of the pair's paths, summed in a fixed
 * order (FP64), with the arguments of sbr_channel (H_c64 and/or H_c128 hold
 * the field to add to: host, or device with SBR_OUT_DEVICE) */
sbr_status sbr_diff_channel(sbr_context_t ctx, sbr_diff_t d, const double* freq_hz, int32_t Nf,
                            const float* atm_db_per_m, const float* atm_deg_per_m, int32_t pol_tx, int32_t pol_rx,
                            void* H_c64, double* H_c128, uint32_t flags);
/* per-path diffracted fields [paths][Nf] interleaved FP64 (diagnostic / parity output) */
sbr_status sbr_diff_field(sbr_context_t ctx, sbr_diff_t d, const double* freq_hz, int32_t Nf,
                          const float* atm_db_per_m, const float* atm_deg_per_m, int32_t pol_tx, int32_t pol_rx,
                          double* a_c128, uint32_t flags);
/* the transition function F(X) = 2j sqrt(X) e^{jX} int_{sqrt X}^inf e^{-j t^2} dt
 * of the diffraction coefficients at X[n] >= 0 (F = 0 at X = 0), interleaved
 * FP64 (diagnostic / parity output) */
sbr_status sbr_utd_transition(sbr_context_t ctx, const double* X, int64_t n, double* F_c128, uint32_t flags);

/* ------------------------------------------------------------------------ */
/* First-order directive diffuse scattering (the scattering coefficient S of
 * the field of a path, eq. (2), and the directive model based on the
 * effective-roughness theory, Sec. II-A-2 and Fig. 3(b); the paper gives no
 * formula).  The single-lobe directive pattern, first order
 * (Tx -> surface tile -> Rx):
 * tiles: triangle t of area A is cut by its barycentric grid into m^2 equal
 * sub-triangles, m = max(1, ceil(sqrt(A / tile_area))); a tile is one
 * sub-triangle (centroid C, area dS = A / m^2), numbered by triangle, then the
 * upward sub-triangles by (i, j), then the downward ones by (i, j).  A path
 * exists when Tx and Rx lie strictly on the same side of the triangle's plane
 * and neither leg crosses a triangle outside the tile's face group (the
 * image-method margins).  Field: the specular reflection of the incidence at
 * C (the faces' Fresnel coefficients, eq. (6)-(7), on the reflection
 * tracker's TE/TM bases) without its component along the scattering
 * direction k_s, carrying the share 1 - rho^2 of the reflected power that the
 * Kirchhoff factor rho (eq. (8)) removes from the specular reflection, spread
 * by the lobe ((1 + cos psi) / 2)^alpha around the specular direction and
 * normalised by its half-space integral F_alpha(theta_i):
 *   a = lambda / (4 pi r_i r_s) sqrt(dS cos theta_i / F_alpha)
 *       sqrt(1 - rho^2) ((1 + cos psi) / 2)^(alpha / 2) (E_s . e_rx)
 *       10^(-g (r_i + r_s) / 20) e^{-j (2 pi f (r_i + r_s) / c + pi phi (r_i + r_s) / 180)}.
 * sbr_scatter: tx_xyz [Nt][3], rx_xyz [Nr][3] FP64 (host, or device with
 * SBR_IN_DEVICE); tile_area > 0 in m^2; 0 <= alpha <= 32; finishes before it
 * returns; the handle keeps the scene.  Errors: INVALID_ARG (NULL, sizes,
 * non-finite points, tile_area or alpha out of range), UNSUPPORTED when
 * tiles x Nt x Nr >= 2^32, there are 2^31 tiles or more, or a triangle
 * would need m >= 65536 (all checked before any tile is made), and when
 * 2^31 paths or more are found. */
sbr_status sbr_scatter(sbr_context_t ctx, sbr_scene_t sc, const double* tx_xyz, int32_t Nt, const double* rx_xyz,
                       int32_t Nr, double tile_area, int32_t alpha, uint32_t flags, sbr_scat_t* out);
/* counts: tiles, (tile, Tx, Rx) candidates, (tile, Tx) and (tile, Rx) legs
 * with the point off the tile's plane and nothing in the way, paths (any
 * output may be NULL) */
sbr_status sbr_scat_info(sbr_scat_t d, int64_t* tiles, int64_t* candidates, int64_t* clear_legs, int64_t* paths);
/* the first min(capacity, paths) paths, ordered by (Rx, Tx, tile), to host
 * arrays: ids [n][3] int32 (tx, rx, tile); rec [n][2] FP64 (r_i = |C - Tx|,
 * r_s = |Rx - C|) */
sbr_status sbr_scat_paths(sbr_scat_t d, int64_t capacity, int32_t* ids, double* rec, int64_t* written);
/* the tiles in their numbering, to host arrays: geo [n][4] FP64 (centroid
 * xyz, area), tri [n] int32 (triangle); count = number of tiles (either
 * output may be NULL) */
sbr_status sbr_scat_tiles(sbr_scat_t d, int64_t capacity, double* geo, int32_t* tri, int64_t* count);
/* H[f][q][p] += the scattered fields of the pair's paths, summed in a fixed
 * order (FP64), with the arguments of sbr_channel (H_c64 and/or H_c128 hold
 * the field to add to: host, or device with SBR_OUT_DEVICE) */
sbr_status sbr_scat_channel(sbr_context_t ctx, sbr_scat_t d, const double* freq_hz, int32_t Nf,
                            const float* atm_db_per_m, const float* atm_deg_per_m, int32_t pol_tx, int32_t pol_rx,
                            void* H_c64, double* H_c128, uint32_t flags);
/* per-path scattered fields [paths][Nf] interleaved FP64 (diagnostic / parity output) */
sbr_status sbr_scat_field(sbr_context_t ctx, sbr_scat_t d, const double* freq_hz, int32_t Nf,
                          const float* atm_db_per_m, const float* atm_deg_per_m, int32_t pol_tx, int32_t pol_rx,
                          double* a_c128, uint32_t flags);
/* the lobe normalisation F_alpha(theta_i) = half-space integral of
 * ((1 + cos psi) / 2)^alpha at cos_i[n] in [0, 1], FP64 (diagnostic / parity
 * output); 0 <= alpha <= 32 */
sbr_status sbr_scatter_lobe_norm(sbr_context_t ctx, int32_t alpha, const double* cos_i, int64_t n, double* out,
                                 uint32_t flags);

/* Per (Rx, Tx) statistics from the path powers of the last sbr_channel:
 * pg_db: 10 log10 sum P_n (incoherent path gain; -inf when no path),
 * tau_rms_s: eq. (5), mean_angles: [Nr][Nt][4] power-weighted (circular mean
 * azimuth, arithmetic mean elevation) of AoD then AoA.  Any output may be
 * NULL.  SBR_E_STATE before sbr_channel. */
sbr_status sbr_stats(sbr_paths_t ps, float* pg_db, float* tau_rms_s, float* mean_angles, uint32_t flags);
/* The same statistics over every mechanism's paths of each (Rx, Tx) link
 * (Table I's quantities from reflection and diffraction paths together):
 * the reflection paths of ps, then, when given, the diffraction paths of d
 * and the scattering paths of sc, each with its band power from its last
 * channel call (sbr_channel, sbr_diff_channel, sbr_scat_channel), its delay
 * (length / c) and its departure and arrival directions (Tx -> first
 * interaction, Rx -> last interaction).  d and sc may be NULL (then the
 * result is sbr_stats's); they must have been made for the same Tx and Rx
 * points, bit for bit.  Errors: SBR_E_STATE before the channel calls,
 * INVALID_ARG for other points or sizes. */
sbr_status sbr_stats_all(sbr_paths_t ps, sbr_diff_t d, sbr_scat_t sc, float* pg_db, float* tau_rms_s,
                         float* mean_angles, uint32_t flags);

/* MIMO capacity, eq. (15)-(17): C(SNR) = band mean of
 * log2 det(I + SNR/Nt W_f), W = Hn Hn^H (Nt >= Nr) or Hn^H Hn (Nt < Nr).
 * normalize = 1: Hn = H sqrt(Nt Nr / Q), Q = band mean of ||H_f||_F^2
 * (the paper's Q scaling read as a Frobenius normalisation); 0: Hn = H.
 * H_c64: [Nf][Nr][Nt] interleaved FP32; snr_db: [Nsnr]; C_bits_per_hz: [Nsnr]
 * FP64.  min(Nr, Nt) <= 128. */
sbr_status sbr_capacity(sbr_context_t ctx, const void* H_c64, int32_t Nf, int32_t Nr, int32_t Nt,
                        const double* snr_db, int32_t Nsnr, int32_t normalize, double* C_bits_per_hz,
                        uint32_t flags);

/* Received power per antenna port pair, eq. (14): h_qp = sqrt(P_qp) e^{i theta_qp}
 * with the paths of (p, q) combined with phase in H (sbr_channel), so
 * P[q][p] = (1/Nf) sum_f |H_f[q][p]|^2, the band mean (FP64; FP32 H entries
 * squared exactly).  The spread of P over the Rx ports of an array is the
 * spatial non-stationarity of Sec. IV-C.  H_c64: [Nf][Nr][Nt] interleaved
 * FP32 (host, or device with SBR_IN_DEVICE; a device H is read in place);
 * P: [Nr][Nt] FP64 (host, or device with SBR_OUT_DEVICE: then the call is
 * queued on the context stream and returns without waiting).  Deterministic:
 * the band is summed in a fixed order. */
sbr_status sbr_port_power(sbr_context_t ctx, const void* H_c64, int32_t Nf, int32_t Nr, int32_t Nt, double* P,
                          uint32_t flags);

/* Allocation-free form of sbr_capacity, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same result as sbr_capacity.
 * H_c64: device pointer [Nf][Nr][Nt] interleaved FP32 on the context's
 * device; C_bits_per_hz: device pointer [Nsnr] FP64; snr_db: host array of
 * Nsnr values (passed to the kernels by value).  Limits: min(Nr, Nt) <= 128,
 * Nsnr <= 64, Nf * (Nsnr + 1) <= 1,048,544 (SBR_E_CAPACITY beyond).  Queued
 * on the context stream without waiting; the work lives in one fixed 8 MiB
 * device array per GPU that every call on that GPU shares, so calls that
 * overlap on one GPU (several streams, threads or contexts) race: order them. */
sbr_status sbr_capacity_noalloc(sbr_context_t ctx, const void* H_c64, int32_t Nf, int32_t Nr, int32_t Nt,
                                const double* snr_db, int32_t Nsnr, int32_t normalize, double* C_bits_per_hz);

/* Launch directions (Sec. II-A-1) for parity checks: dirs [count][3] FP64 of
 * ray ids first .. first+count-1; and the edge-angle statistics (radians) of
 * the geodesic triangulation (any output may be NULL). */
sbr_status sbr_geodesic(sbr_context_t ctx, int32_t N, int64_t first, int64_t count, double* dirs, uint32_t flags);
sbr_status sbr_geodesic_alpha(sbr_context_t ctx, int32_t N, double* mean, double* min, double* max);

/* Scene queries: face group and plane id of every triangle (host [T]). */
sbr_status sbr_scene_info(sbr_scene_t s, int32_t* n_groups, int32_t* n_planes, int32_t* bvh_depth);
sbr_status sbr_scene_groups(sbr_scene_t s, int32_t* group, int32_t* plane);

/* Live per-kernel timing (measurement support, not part of the method).
 * When enabled, the library records a pair of HIP events on the context
 * stream around every kernel launch it makes and accumulates the elapsed time
 * per kernel class ("bounce", "replay_capture", "rebuild", "channel", "sort",
 * "bvh", "keys", "stats", "capacity", "alpha", "misc").  Enabling clears the
 * totals; a query synchronises the stream.  Unknown names report 0. */
sbr_status sbr_profile_enable(sbr_context_t ctx, int enable);
/* Restrict the live timing to one kernel class (its launches only, no host
 * phases), so that measuring one kernel adds two event records per launch of
 * that class and nothing else; NULL or "" times every class again.  Clears
 * the totals.  Unknown names time nothing. */
sbr_status sbr_profile_only(sbr_context_t ctx, const char* kernel);
sbr_status sbr_profile_query(sbr_context_t ctx, const char* kernel, double* total_ms, int64_t* launches);
/* Traversal work counters: with counting enabled (sbr_context_count_work),
 * later traces also count BVH node visits and ray-triangle tests of the
 * closest-hit search; sbr_trace_work returns them (0 when not counted). */
sbr_status sbr_context_count_work(sbr_context_t ctx, int enable);
sbr_status sbr_trace_work(sbr_trace_t tr, int64_t* node_visits, int64_t* tri_tests);

/* Launch tuning (see the autotuner in the Python package).  Keys:
 *   "trace_blocks_per_cu"  resident 256-thread blocks per CU of the persistent
 *                          bounce grid (1..32, default 4)
 *   "trace_chunk"          rays a wave takes from its queue per atomic (multiple of 64, <= 4096)
 *   "trace_leaf_share"     leaves found during the closest-hit traversal wait until
 *                          this many 64ths of the wave's tracing lanes hold one (or
 *                          no lane can go on without a test) and are then tested
 *                          together (1..64, default 40; 1: every traversal step
 *                          tests the leaves it found)
 *   "replay_block"         threads per block of the capture replay (64..1024, a multiple
 *                          of 64); a receive lowers it in whole waves when the
 *                          traversal stacks of a block (deep receiver trees) would
 *                          not fit 64 KiB of LDS
 *   "trace_graph"          1: the bounce loop of sbr_trace runs as a hipGraph built
 *                          once per (bounces, tree depth class) and replayed with
 *                          updated kernel arguments; 0 (default): direct launches
 *   "bvh_ploc_max"         scenes built later with up to this many triangles get a
 *                          PLOC-clustered BVH, larger ones the Morton-ordered LBVH
 *                          with an oversized-triangle list (0..65536, default 65536)
 *   "trace_order"          1 (default): traces of several Tx elements keep their rays
 *                          element-minor (neighbouring lanes follow one launch
 *                          direction from neighbouring elements); 0: element-major.
 *                          Results are the same either way
 *   "trace_packet"         1: the closest-hit search of a (single-scene) trace walks
 *                          the tree once per wave, entering a node when any of the
 *                          wave's rays enters it; 0 (default): every ray walks it on
 *                          its own.  The hits are the same either way; traces that
 *                          count work and batched traces always walk per ray
 *   "receive_event_capacity"  first size of the capture-event buffer of a receive
 *                          (>= 0; 0, the default: max(2^20, rays / 8)); a receive
 *                          that overflows it grows it and replays again
 * Unknown keys or out-of-range values: SBR_E_INVALID_ARG. */
sbr_status sbr_context_set_tuning(sbr_context_t ctx, const char* key, int32_t value);
sbr_status sbr_context_get_tuning(sbr_context_t ctx, const char* key, int32_t* value);

/* Release any handle (context, scene, trace, paths); NULL is ignored. */
void sbr_release(void* handle);
const char* sbr_last_error(void);
const char* sbr_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SBR_H_ */

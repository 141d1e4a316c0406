/*
 * gi.h -- C ABI of the MI355X (gfx950) implementation of the per-frame indirect-lighting
 * pass of GI-1.0 (Boisse et al. 2022, "GI-1.0: A Fast Scalable Two-Level Radiance Caching
 * Scheme for Real-Time Global Illumination").
 *
 * The pass (Section 2): screen-space probes, one per 8x8 pixel tile, trace rays over their
 * oriented hemisphere (screen cache, Section 2.1); every ray hit reads and fills a
 * world-space spatial-hash radiance cache (world cache, Section 2.2); the probes are
 * projected to spherical harmonics and interpolated per pixel (Section 2.4).  A learned
 * surrogate of the world cache (multiresolution hash encoding + small MLP, trained online on
 * the samples the pass produces) can replace the cell lookups at probe-ray hits.
 *
 * Conventions (every entry point):
 *   - Return value: GI_OK (0) or a negative gi_status.  No C++ exception crosses the ABI.
 *     The text of the last error of a context is kept until the next call on it
 *     (gi_last_error).
 *   - Pointers named d_* are device pointers (hipMalloc'd or torch-owned memory on the
 *     context's device); pointers named h_* are host pointers.  The caller owns every pointer
 *     it passes; device pointers must stay valid until the work queued on `stream` is done.
 *     Device pointers must be 16-byte aligned.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Per-frame calls only enqueue
 *     work and return; gi_build_bvh, the export / import calls and gi_get_stats synchronise.
 *   - The context owns all internal buffers (BVH, world cache, probes, ray records, learned
 *     cache state) and frees them in gi_destroy.  A context is used by one host thread at a
 *     time.
 *   - Frame order: gi_spawn_probes -> gi_trace_probes -> [gi_learned_train] ->
 *     gi_cache_update -> gi_interpolate_probes.  Calls out of order return GI_ERR_STATE.
 *   - Results are deterministic: every integer result (probe mask, hit index, hit distance
 *     bits, cell key, per-cell fixed-point sums and counts) is bit-reproducible and equal to
 *     the float32 definition of the method; the slot a cell occupies inside its bucket is not
 *     part of the result, so exports list cells in ascending key order.
 */
#ifndef GI_H
#define GI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gi_status;
enum {
    GI_OK = 0,
    GI_ERR_INVALID_ARG = -1,  /* null / misaligned pointer, size or config out of range */
    GI_ERR_OOM = -2,          /* device or host allocation failed */
    GI_ERR_HIP = -3,          /* a HIP runtime call failed */
    GI_ERR_STATE = -4,        /* call out of frame order, or before gi_build_bvh */
    GI_ERR_UNSUPPORTED = -5,  /* device is not gfx950, or a feature the library does not provide */
    GI_ERR_INTERNAL = -6      /* unexpected failure (message in gi_last_error) */
};

enum { GI_CACHE_PLAIN = 0, GI_CACHE_MLP_BF16 = 1, GI_CACHE_MLP_FP8 = 2 };

/* ray-record flag bits (gi_rays_export): bits 0..5 hemisphere cell of the probe atlas */
#define GI_RAY_HIT 0x100u     /* the probe ray hit a triangle */
#define GI_RAY_FRONT 0x200u   /* ... on the side its winding normal faces (emission side) */
#define GI_RAY_EMIT 0x400u    /* ... on that side of a triangle whose material emits */
#define GI_RAY_TRACED 0x10000u

/* interpolation flag (alpha of gi_interpolate_probes output) */
#define GI_INTERP_OK 0.0f
#define GI_INTERP_RELAXED 1.0f   /* all weights zero: equal weights (Section 2.4.1) */
#define GI_INTERP_NO_PROBE 2.0f  /* no neighbour probe found */
#define GI_INTERP_SKY 3.0f

typedef struct gi_config {
    uint32_t width, height;      /* G-buffer size in pixels (>= 8 each, <= 8192)          */
    uint32_t rays_per_probe;     /* R, 1..256 (Section 2.1: rays per 8x8 probe)           */
    uint32_t table_log2;         /* world-cache slots N = 2^table_log2, 6..28            */
    uint32_t bounces;            /* 1: one light sample per hit; 2: + one cached bounce   */
    uint32_t leak_bit;           /* add (ray length < cell size) to the descriptor (2.2.2) */
    uint32_t max_life;           /* accesses keep a cell alive this many idle updates     */
    uint32_t n_cap;              /* moving-average history cap in samples (0 = replace)   */
    uint32_t seed;               /* seed of the counter-based random streams              */
    uint32_t frac_bits;          /* fixed-point fraction bits F of cell sums (1..16)       */
    uint32_t cache_mode;         /* GI_CACHE_*                                            */
    uint32_t probe_filter;       /* 1: separable 7x7 probe-space filter (Algorithm 5) before SH */
    float cell_scale;            /* S = 1 / cell size of the position quantiser (2.2.1)    */
    float r_max;                 /* clamp of a cache sample before quantisation; with
                                    frac_bits: r_max * 2^F * 64 < 2^32 (a wave's group sum
                                    of one cell fits a u32), else GI_ERR_INVALID_ARG      */
    float eps_scale;             /* ray origin offset = eps_scale * (1 + max|p_i|)        */
    float t_sky;                 /* travelled distance recorded for a ray that misses     */
    float sky[4];                /* environment radiance returned by a miss (rgb, pad)    */
    /* learned surrogate of the world cache (used when cache_mode != GI_CACHE_PLAIN) */
    uint32_t mlp_batch_log2;     /* training samples per frame = 2^mlp_batch_log2 (<= 20)  */
    uint32_t mlp_levels;         /* hash-grid levels (<= 16)                              */
    uint32_t mlp_table_log2;     /* entries per level = 2^mlp_table_log2 (<= 22)          */
    uint32_t mlp_steps;          /* optimiser steps per frame                             */
    float mlp_lr_grid, mlp_lr_mlp;
    float mlp_loss_scale;        /* static loss scale                                     */
    float mlp_judge;             /* max rel. error vs confident plain cells before fallback */
    float scene_min[4], scene_max[4];  /* encoding domain (set by gi_build_bvh if zero)   */
    /* levels of detail of the world cache (Section 2.2.1): at a hit d metres from the camera
     * of the frame's spawn, cells are 2^lod times the base size, lod the smallest integer
     * (<= 7) with 2^lod >= lod_scale * d * cell_scale, and lod enters the descriptor (bits
     * 58-60).  lod_scale = Algorithm 6's distance scale keeps world cells about the size of the
     * screen cache's adaptive cell; 0 = a single level. */
    float lod_scale;
    /* 1: temporal reuse of screen probes (Section 2.1.1, Algorithm 1: a tile whose previous
     * probe reprojects onto one of its pixels keeps it there; Section 2.1.4, Algorithm 3: its
     * new radiance is blended with that history). */
    uint32_t temporal;
    /* temporal upscaling (Section 2.1.1 spawn tiles, Section 2.1.2 Algorithm 2), 0 or 1 =
     * off, 2..4 = u (needs temporal = 1): a spawn tile is u x u probe tiles and the frame's
     * Halton jitter in [0, 8u)^2 picks one pixel in it; only the probe tile holding that pixel
     * (if not sky) traces new rays.  Tiles whose probe reprojected keep it, traced or not
     * (untraced ones keep their history radiance); a tile with neither takes the rays of a
     * randomly picked tile that is both (adaptive sampling), the lowest-numbered of several
     * such takers winning.  About 1/u^2 of the rays of upscale 1. */
    uint32_t upscale;
    /* 1: ray guiding (Section 2.1.2; needs temporal = 1).  Each new probe's hemisphere is
     * reconstructed from the previous probes of the 3x3 tiles around its projection that pass
     * the reprojection's plane and normal tests, parallax-corrected through their travelled
     * distances; rays pick cells in proportion to the reconstruction's luminance (integer
     * inverse CDF) and a uniform point inside the cell.  The reconstruction is the history
     * of Algorithm 3 and the radiance of probes kept without tracing. */
    uint32_t ray_guiding;
    /* 1: two-level world cache (Section 2.2.3; plain cache_mode only).  The hash table holds
     * 2^table_log2 tiles instead of cells; a tile covers 8x8x8 cells of the descriptor's grid
     * (position quantised, divided by 8) and stores 8x8 2D cells: the remainders modulo 8 of
     * the two axes other than the main axis of the normal class.  Each update takes the
     * moving average of every cell, rebuilds MIP levels 4x4, 2x2, 1x1 as sample-weighted
     * means of 2x2 children, and every reader (probe rays, bounces, gi_cache_query) sees the
     * finest of the cell's level and its parents holding at least tile_min_samples samples
     * (else the coarsest level if it holds any).  Export with gi_tiles_export. */
    uint32_t cache_tiles;
    uint32_t tile_min_samples;
    /* 1: light sampling by RIS over a light grid (Section 2.3).  After the probe rays, a grid
     * of cubic cells (longest axis in lgrid_dim cells, 1..32) is laid over the box of the
     * frame's hit points; each cell keeps the lgrid_k (1..256) emitter triangles of largest
     * importance (mean over its corners of luminance * area * cos / max(d^2, area)), lights
     * facing away from the cell or farther than sqrt(luminance * area / lgrid_threshold)
     * culled.  Each hit draws ris_candidates (1..8) candidates from its cell's list (a
     * uniform pick, a uniform point) and keeps one by weighted reservoir sampling with target
     * luminance * cos * cos / d^2; one shadow ray.  At most 2048 emitter triangles. */
    uint32_t light_grid;
    uint32_t ris_candidates;
    uint32_t lgrid_dim;
    uint32_t lgrid_k;
    float lgrid_threshold;
    /* 1: world-space reservoir reuse (Section 2.3.1; needs light_grid).  Each hit's final
     * reservoir (light point, contribution weight, count, its normal) is kept in a spatial
     * hash over the quantised position alone (2^restir_log2 slots, 6..24; per cell the
     * lowest ray id's); the next frame, a hit whose cell holds one with a normal cosine above
     * 0.9 resamples it into its own reservoir, its count capped at restir_cap (1..64) x
     * ris_candidates. */
    uint32_t restir;
    uint32_t restir_log2;
    uint32_t restir_cap;
} gi_config;

typedef struct gi_frame {
    uint32_t index;              /* frame number (jitter and random streams)              */
    float fov_y;                 /* vertical field of view, radians                       */
    float tan_half;              /* tan(fov_y / 2) as float32                             */
    float pad;
    float pos[4], fwd[4], right[4], up[4];   /* camera position and orthonormal basis     */
} gi_frame;

typedef struct gi_context gi_context;

/* Stats counters (gi_get_stats), cumulative since creation or gi_reset_stats */
enum {
    GI_STAT_RAYS = 0, GI_STAT_HITS, GI_STAT_INSERTS, GI_STAT_OVERFLOW, GI_STAT_NONFINITE,
    GI_STAT_WRAPS, GI_STAT_SHADOW, GI_STAT_OCCLUDED, GI_STAT_EVICT, GI_STAT_LIVE,
    GI_STAT_RELAXED, GI_STAT_NOPROBE, GI_STAT_BOUNCE, GI_STAT_MLP_SKIPPED, GI_STAT_MLP_FALLBACK,
    GI_STAT_COUNT = 16
};

/* ---- lifetime ------------------------------------------------------------------------- */

/* Create a context on the current HIP device with a copy of *cfg.  Validates the config and
 * that the device is gfx950; allocates the world cache, probe and ray buffers. */
gi_status gi_create(const gi_config *cfg, gi_context **out);
void gi_destroy(gi_context *ctx);
const char *gi_last_error(const gi_context *ctx);
/* Library version string and the offload target it was built for. */
const char *gi_version(void);

/* ---- scene ---------------------------------------------------------------------------- */

/* Build the ray-tracing acceleration structure on the host (binned-SAH binary tree with
 * spatial splits, collapsed to a 4-wide BVH, nodes of one 128-byte line, triangles in leaf
 * order; a triangle split in space fills several leaf slots) and upload it,
 * together with unit triangle normals, materials and the area-proportional emitter table.
 * h_verts [n_verts][3] float; h_idx [n_tris][3]; h_tri_mat [n_tris]; h_mats [n_mats][6]
 * (albedo rgb, emitted radiance rgb).  Synchronous.  The paper traverses with hardware
 * (Section 4); any traversal returning the closest hit serves the method. */
gi_status gi_build_bvh(gi_context *ctx, const float *h_verts, uint32_t n_verts,
                       const uint32_t *h_idx, uint32_t n_tris, const uint32_t *h_tri_mat,
                       const float *h_mats, uint32_t n_mats);

/* Host only (no context, no device): the 4-wide BVH that gi_build_bvh builds, for inspection
 * and tests.  h_tri_verts [n_tris][9] float: the vertex positions of each triangle.
 * A node record is 128 bytes: child boxes as float[4] each of lo x, hi x, lo y, hi y, lo z,
 * hi z, then uint32 child[4] (an inner node index; a leaf 0x80000000 | (count - 1) << 24 |
 * first leaf slot; 0xFFFFFFFF empty), then 16 bytes of padding.  Node 0 is the root, always
 * an inner node.  Leaf slots hold triangle indices.  *n_nodes, *n_slots and *depth (levels
 * of the 4-wide tree) are always set; h_nodes (cap_nodes records) and h_slots (cap_slots
 * entries) are filled when not null, and a capacity smaller than the result is
 * GI_ERR_INVALID_ARG.  GI_ERR_OOM if host memory runs out. */
gi_status gi_bvh_build_host(const float *h_tri_verts, uint32_t n_tris, void *h_nodes, uint32_t cap_nodes,
                            uint32_t *h_slots, uint32_t cap_slots, uint32_t *n_nodes, uint32_t *n_slots,
                            uint32_t *depth);

/* Replace the set of moving triangles tested beside the BVH (at most 64): h_tri_verts
 * [n][9] float, h_tri_mat [n].  Their indices follow the static ones.  Rebuilds the emitter
 * table; enqueued on `stream`. */
gi_status gi_set_dynamic_triangles(gi_context *ctx, const float *h_tri_verts,
                                   const uint32_t *h_tri_mat, uint32_t n, void *stream);

/* Primary visibility (the G-buffer the paper rasterises, Section 2.1.1): one ray through
 * every pixel centre.  d_pos [H][W][4] (hit point, view distance), d_nrm [H][W][4]
 * (face-forwarded unit normal), d_alb [H][W][4], d_prim [H][W] (triangle or 0xFFFFFFFF). */
gi_status gi_render_gbuffer(gi_context *ctx, const gi_frame *frame, float *d_pos, float *d_nrm,
                            float *d_alb, uint32_t *d_prim, void *stream);

/* ---- the per-frame pass --------------------------------------------------------------- */

/* Section 2.1.1 and 2.1.5: one probe per 8x8 tile at the frame's Halton-jittered pixel
 * (sentinel if off screen or sky), its position and normal from the G-buffer, the probe
 * mask and its MIP chain (first valid probe of each 2x2 block). */
gi_status gi_spawn_probes(gi_context *ctx, const gi_frame *frame, const float *d_pos,
                          const float *d_nrm, const uint32_t *d_prim, void *stream);

/* Sections 2.1.3, 2.2.1-2.2.4, 2.3.1: R cosine-distributed rays per probe, closest hit;
 * every hit looks up or creates its world-cache cell (bucket by a PCG hash, fingerprint by
 * XXH32, linear probing inside a 32-slot bucket) and adds one fixed-point radiance sample:
 * one area-sampled light point with one shadow ray, plus (bounces = 2) the cached radiance at
 * the end of one cosine bounce ray. */
gi_status gi_trace_probes(gi_context *ctx, const gi_frame *frame, void *stream);

/* Sections 2.2.1, 2.2.3, 2.1.4, 2.4.2: per cell, the frame's mean sample enters the
 * moving average and the decay counter is updated (cells idle for max_life updates are
 * freed); per probe, ray radiance is averaged per atlas cell, empty cells get the mean of
 * the populated ones, and the atlas is projected onto 9 SH coefficients per channel. */
gi_status gi_cache_update(gi_context *ctx, const gi_frame *frame, void *stream);

/* Section 2.4.1 with Algorithms 4 and 6: per-pixel irradiance from the 2x2 neighbour probes
 * (edge-aware weights, relaxed fallback).  d_out [H][W][4]: rgb irradiance, alpha = flag. */
gi_status gi_interpolate_probes(gi_context *ctx, const gi_frame *frame, const float *d_pos,
                                const float *d_nrm, const uint32_t *d_prim, float *d_out,
                                void *stream);

/* Lookup-only read of the world cache (Section 2.1.3: a hit's radiance from its cell).
 * d_pos [n][4] (xyz, w = ray length for the leak bit or < 0 for none), d_nrm [n][4];
 * d_out [n][4]: cached radiance rgb, alpha 1 if the cell exists, else 0. */
gi_status gi_cache_query(gi_context *ctx, const float *d_pos, const float *d_nrm, uint32_t n,
                         float *d_out, void *stream);

/* Traversal only (tests and measurement): d_o [n][4], d_d [n][4] (w of d_o = tmax);
 * closest hit (d_tri, d_t) or, with any_hit, d_tri[i] = 1 if anything lies in (0, tmax). */
gi_status gi_trace_rays(gi_context *ctx, const float *d_o, const float *d_d, uint32_t n,
                        uint32_t any_hit, uint32_t *d_tri, float *d_t, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): gi_trace_rays with the same arguments and
 * results (bit-identical), whose traversal-stack spill rows live in a fixed 16 MiB device
 * array, one per GPU, held from library load until the process ends, instead of the
 * context's spill buffer.  It calls no allocator.  The context must have been created on the
 * current device (its gi_create looked up the array's address there; else
 * GI_ERR_INVALID_ARG).  Rays go in chunks of (4 Mi / spill rows) lane ids, rounded down to
 * 64; a BVH too deep for one chunk of 64 (more than 65,536 spill rows, which gi_build_bvh
 * never produces) is GI_ERR_UNSUPPORTED.  Every call on one GPU shares that GPU's array:
 * calls that overlap in time on one GPU (other streams, other threads, other contexts) race
 * and give undefined results; serialise them. */
gi_status gi_trace_rays_noalloc(gi_context *ctx, const float *d_o, const float *d_d, uint32_t n,
                                uint32_t any_hit, uint32_t *d_tri, float *d_t, void *stream);

/* Measurement: re-walk the last traced frame's probe rays and their shadow rays with an
 * instrumented copy of the traversal (no other side effect).  h_out8: [0] probe rays,
 * [1] nodes visited, [2] triangles tested, [3] shadow rays, [4] nodes, [5] triangles.
 * Call after gi_trace_probes; synchronises. */
gi_status gi_measure_traversal(gi_context *ctx, uint64_t *h_out8, void *stream);

/* ---- learned radiance-cache surrogate (not in the paper) ------------------------------ */

/* Select mlp_steps * 2^mlp_batch_log2 of this frame's hit samples (stratified over the hits)
 * and take mlp_steps optimiser steps of 2^mlp_batch_log2 samples each, step k on every
 * mlp_steps-th of them (hash-grid + MLP forward, relative-L2 loss, backward, Adam) with the
 * library's kernels.  Between gi_trace_probes and gi_cache_update.  GI_ERR_STATE in plain
 * mode. */
gi_status gi_learned_train(gi_context *ctx, const gi_frame *frame, void *stream);

/* One optimiser step on caller samples (tests, warm starts): d_pos, d_nrm, d_target [n][4]
 * with n == 2^mlp_batch_log2.  apply = 0 computes the gradients only (kept for
 * gi_learned_save), apply = 1 also takes the Adam step. */
gi_status gi_learned_step(gi_context *ctx, const float *d_pos, const float *d_nrm, const float *d_target,
                          uint32_t n, uint32_t apply, void *stream);

/* The OCP e4m3 code (round to nearest even, saturating to +-448, NaN -> 0x7F) that FP8
 * inference gives its weights and activations after scaling: d_in [n] floats -> d_out [n]
 * bytes.  Exposed so that the encoder can be checked against a reference codec. */
gi_status gi_e4m3_encode(gi_context *ctx, const float *d_in, uint8_t *d_out, uint32_t n, void *stream);

/* Evaluate the surrogate at caller points: d_pos [n][4], d_nrm [n][4] -> d_out [n][4]. */
gi_status gi_learned_query(gi_context *ctx, const float *d_pos, const float *d_nrm, uint32_t n,
                           float *d_out, void *stream);

/* ---- screen-space denoiser (Section 2.4.3) ------------------------------------------------
 * A separate object: it needs the G-buffer, the interpolated irradiance and the camera only.
 * Temporal accumulation over the reprojected history (valid when the previous pixel held one,
 * was not sky, lies within the pixel's cell size of its tangent plane and has a normal cosine
 * above 0.9): history length n = min(n + 1, hist_max) (1..1024), value = history + (E -
 * history) / n; otherwise n = 1.  Pixels without a probe (flag 2) keep their history.  Then a
 * spatial filter of radius floor(radius_max / n) (0..16; radius_max at n = 0) dilated over the
 * 3x3 neighbourhood, weights cs / (cs + |depth difference|) * max(0, normal cosine)^8.  The
 * accumulated values before the filter are the next frame's history. */
typedef struct gi_denoiser gi_denoiser;
gi_status gi_denoiser_create(uint32_t width, uint32_t height, uint32_t hist_max, uint32_t radius_max,
                             gi_denoiser **out);
void gi_denoiser_destroy(gi_denoiser *dn);
/* forget the history (the next frame starts over) */
gi_status gi_denoiser_reset(gi_denoiser *dn);
/* device pointers owned by the caller, 16-byte aligned: the G-buffer of gi_render_gbuffer
 * (pos [H][W][4] with w = view distance, nrm [H][W][4], prim [H][W]), the irradiance of
 * gi_interpolate_probes [H][W][4] (rgb, flag) -> out [H][W][4] (rgb, the same flag); async on
 * stream; calls on one denoiser are serialised by the caller */
gi_status gi_denoise(gi_denoiser *dn, const gi_frame *frame, const float *d_pos, const float *d_nrm,
                     const uint32_t *d_prim, const float *d_irradiance, float *d_out, void *stream);
/* host-synchronous: the history (rgb, n) [H][W][4] and the radius per pixel [H][W] */
gi_status gi_denoiser_export(gi_denoiser *dn, float *h_hist, uint32_t *h_radius);

/* ---- parity, resume and observability (host-synchronous, host pointers) --------------- */

/* Two-level cache export (cache_tiles = 1; host-synchronous): the live tiles in ascending key order,
 * at most cap of them; id = bucket << 32 | fingerprint, key = tile descriptor, life, and per
 * cell (64 per tile, [n][64][...]) the fixed-point sums and count of this frame, the moving
 * average, its sample count and the prefiltered radiance that readers see.  Any output
 * pointer may be null.  GI_ERR_UNSUPPORTED without tiles. */
gi_status gi_tiles_export(gi_context *ctx, uint64_t *h_id, uint64_t *h_key, uint32_t *h_life, uint32_t *h_acc,
                          float *h_L, uint32_t *h_nhist, float *h_Lq, uint32_t cap, uint32_t *n_out);

/* Light grid of the last trace (light_grid = 1; host-synchronous): geom = origin x, y, z and
 * cell side; dims = cells per axis; per cell (x fastest, at most cap_cells) the emitter
 * indices (into the emitter order: static emitters in triangle order, then dynamic ones;
 * lgrid_k per cell, the first count[c] valid) and the count.  GI_ERR_UNSUPPORTED without it. */
gi_status gi_light_grid_export(gi_context *ctx, float *h_geom, uint32_t *h_dims, uint32_t *h_list, uint32_t *h_count,
                               uint32_t cap_cells);

/* World-space reservoirs written by the last trace (restir = 1; host-synchronous): live slots
 * in ascending key order, at most cap: id = bucket << 32 | fingerprint, key (quantised position),
 * light point and contribution weight [n][4], normal of the storing vertex [n][3], light
 * (emitter index) and count.  GI_ERR_UNSUPPORTED without reservoirs. */
gi_status gi_restir_export(gi_context *ctx, uint64_t *h_id, uint64_t *h_key, float *h_yw, float *h_n, uint32_t *h_k,
                           uint32_t *h_m, uint32_t cap, uint32_t *n_out);

/* Live cells in ascending key order: id = bucket << 32 | fingerprint, key (descriptor bits), acc
 * [n][4] (fixed-point r,g,b sums and count of the current frame), L [n][3] cached radiance,
 * nhist, life.  Writes at most cap cells; *n_out = number of live cells.
 * GI_ERR_UNSUPPORTED with cache_tiles (see gi_tiles_export); so are save and load. */
gi_status gi_cache_export(gi_context *ctx, uint64_t *h_id, uint64_t *h_key, uint32_t *h_acc,
                          float *h_L, uint32_t *h_nhist, uint32_t *h_life, uint32_t cap,
                          uint32_t *n_out);

/* Whole world-cache state as an opaque blob (resume): *size_out bytes; h_blob NULL queries
 * the size only.  gi_cache_import restores a blob from a context of the same config. */
gi_status gi_cache_save(gi_context *ctx, void *h_blob, size_t cap, size_t *size_out);
gi_status gi_cache_load(gi_context *ctx, const void *h_blob, size_t size);
/* The same as gi_cache_load: restore a world cache saved from a context of the same config. */
gi_status gi_cache_import(gi_context *ctx, const void *h_blob, size_t size);

/* Ray records of the last gi_trace_probes, [P*R] each: slot (or -1), t, tri, flags; and the
 * descriptor key of the hit (0 for a miss). */
gi_status gi_rays_export(gi_context *ctx, int32_t *h_slot, float *h_t, uint32_t *h_tri,
                         uint32_t *h_flags, uint64_t *h_key);

/* Probe state: mask with all MIP levels concatenated (level 0 first), probe pos / normal
 * [P][4], atlas [P][64][4] (rgb, mean hit distance), SH [P][27] (9 coefficients x rgb).
 * Any pointer may be NULL. */
gi_status gi_probes_export(gi_context *ctx, uint32_t *h_mask, float *h_pos, float *h_nrm,
                           float *h_atlas, float *h_sh);

/* Sizes: [0] P, [1] R, [2] N, [3] TW, [4] TH, [5] MIP levels, [6] mask entries (all
 * levels), [7] jitter x, [8] jitter y, [9] BVH nodes, [10] BVH depth. */
gi_status gi_get_dims(gi_context *ctx, uint32_t *h_out16);
gi_status gi_get_stats(gi_context *ctx, uint64_t *h_out16);
gi_status gi_reset_stats(gi_context *ctx, void *stream);

/* Per-kernel device timing with HIP events on the launch stream: on = 1 times every kernel,
 * on = 2 only the probe-ray traversal (two events per frame, so a measured run stays as it
 * is), 0 none; other values are GI_ERR_INVALID_ARG.  The events skip the system-scope fence.
 * Read returns, for up to cap kernels, NUL-separated names, launch counts and total ms since
 * the last read, and resets the totals.  Reading synchronises. */
gi_status gi_profile_enable(gi_context *ctx, uint32_t on);
gi_status gi_profile_read(gi_context *ctx, char *h_names, size_t names_cap, uint32_t *h_counts,
                          double *h_ms, uint32_t cap, uint32_t *n_out);

/* Learned-cache parameters as a blob (resume); layout private to the library. */
gi_status gi_learned_save(gi_context *ctx, void *h_blob, size_t cap, size_t *size_out);
gi_status gi_learned_load(gi_context *ctx, const void *h_blob, size_t size);
/* The same as gi_learned_save / gi_learned_load (the surrogate's parameters, gradients and
 * Adam state as one blob; import requires a context of the same levels and table size). */
gi_status gi_learned_export(gi_context *ctx, void *h_blob, size_t cap, size_t *size_out);
gi_status gi_learned_import(gi_context *ctx, const void *h_blob, size_t size);
/* The last gi_learned_train's batch (host-synchronous; learned mode).  The frame's training
 * rays are the probe rays whose hit found or created a world-cache cell with a finite sample,
 * in ray order (ray id = probe * R + ray); the batch's rows = mlp_steps * 2^mlp_batch_log2
 * (at most 2^20) picks, pick k = training ray floor((k + u) * n / rows) with n the number of
 * training rays and u the frame's uniform number of the seeded stream (frame, id 2^31 - 1,
 * dimension 9).  h_raw [rows][12] floats in pick order: hit point and distance, face-forwarded
 * normal with the ray id's bits in the 4th float, training target rgb and 1; h_grouped the
 * same rows stably sorted by the 15-bit Morton code of the position normalised to the
 * encoding domain (32 cells per axis): optimiser step k trains on grouped rows k, k + s,
 * k + 2s, ... with s = rows / 2^mlp_batch_log2.  *rows_out and *n_train_out are always set;
 * the arrays (either may be NULL) are filled when cap_rows >= rows, else GI_ERR_INVALID_ARG. */
gi_status gi_learned_batch_export(gi_context *ctx, float *h_raw, float *h_grouped, uint32_t cap_rows,
                                  uint32_t *rows_out, uint32_t *n_train_out);

/* Loss of the last training step and the fallback decision of the last update:
 * [0] loss, [1] judged relative error, [2] fallback (0/1), [3] steps taken, [4] steps skipped */
gi_status gi_learned_stats(gi_context *ctx, float *h_out8);

#ifdef __cplusplus
}
#endif
#endif /* GI_H */

/*
 * pt.h -- C ABI of the MI355X path tracer (libpt.so, HIP for gfx950).
 *
 * The library estimates, per pixel, the Monte Carlo integral of the
 * rendering equation (paper Sec. 1.1): camera rays (Sec. 5.1.2), closest
 * hits through a BVH of axis-aligned boxes built on the CPU (Sec. 5.1.1),
 * OpenPBR surface shading with importance sampling and Russian roulette
 * (Sec. 4, Sec. 5.1.3), next-event estimation with multiple importance
 * sampling, and per-pixel averaging of the samples (Sec. 5.1.3).  The paper
 * splits the work into a CPU set-up done once per scene and GPU sampling
 * repeated per frame (Sec. 5.1); the calls below follow that split.
 *
 * Conventions
 *  - Every call returns pt_status and never throws.  On error the scene is
 *    left unchanged and pt_last_error() (thread-local) explains why.
 *  - Host input arrays are copied during the call; the caller keeps
 *    ownership and may free them on return.
 *  - Device pointers (out_rgb32f, rays, hits, ...) are caller-owned memory
 *    on the scene's device, allocated for example as torch tensors.
 *  - Work is enqueued on the scene's stream; calls that return results
 *    synchronise that stream before returning, so device faults surface as
 *    PT_ERR_DEVICE.
 *  - Output radiance is linear RGB; row 0 is the top of the image.
 *  - No call is safe to run concurrently on the same scene.
 */
#ifndef PT_H
#define PT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum pt_status {
  PT_OK = 0,
  PT_ERR_INVALID_ARG = -1,  /* a pointer, count, index or parameter is out of range */
  PT_ERR_OUT_OF_MEMORY = -2,
  PT_ERR_DEVICE = -3,       /* a HIP call failed (message has the HIP error string) */
  PT_ERR_UNSUPPORTED = -4,  /* a valid parameter combination this library does not implement */
  PT_ERR_STATE = -5         /* e.g. render before pt_build_bvh / pt_upload_materials */
} pt_status;

typedef struct pt_scene pt_scene; /* opaque; owns every device allocation it makes */

/* A triangle mesh (host pointers).  Triangles are the paper's geometry
 * (Sec. 5.1.1); winding defines the front face: the geometric normal is
 * normalize(cross(v1 - v0, v2 - v0)).  Zero-area triangles are accepted and
 * never hit. */
typedef struct pt_mesh {
  const float* vertices;        /* [n_vertices][3], finite */
  int64_t n_vertices;
  const int32_t* indices;       /* [n_triangles][3], each in [0, n_vertices) */
  int64_t n_triangles;          /* >= 1 */
  const int32_t* material_ids;  /* [n_triangles]; may be NULL if every instance overrides */
} pt_mesh;

/* A placement of a mesh (two-level hierarchy).  object_to_world is a
 * row-major 3x4 rigid transform (rotation | translation). */
typedef struct pt_instance {
  float object_to_world[12];
  int32_t mesh;
  int32_t material_override;  /* -1: use the mesh's per-triangle ids */
} pt_instance;

/* OpenPBR parameters (Sec. 4), linear RGB; 39 floats in this order.
 * thin_film_thickness is in micrometres.  Subsurface is its local limit: a
 * diffuse reflector of albedo subsurface_color mixed into the dielectric
 * base by subsurface_weight (no light travels sideways under the surface,
 * so OpenPBR's subsurface radius and anisotropy are not parameters). */
typedef struct pt_openpbr_material {
  float base_weight, base_color[3], base_metalness, base_diffuse_roughness;
  float specular_weight, specular_color[3], specular_roughness, specular_roughness_anisotropy,
      specular_ior;
  float transmission_weight, transmission_color[3];
  float coat_weight, coat_color[3], coat_roughness, coat_ior;
  float emission_luminance, emission_color[3];
  float thin_film_weight, thin_film_thickness, thin_film_ior;
  float fuzz_weight, fuzz_color[3], fuzz_roughness;
  float subsurface_weight, subsurface_color[3];
} pt_openpbr_material;

/* Pinhole camera (Sec. 5.1.2): vertical field of view in degrees, aspect width/height. */
typedef struct pt_camera {
  float eye[3], look_at[3], up[3];
  float vfov_deg;
  int32_t width, height;
} pt_camera;

typedef struct pt_stats {
  int64_t extension_rays;    /* closest-hit rays traced since the last reset */
  int64_t shadow_rays;       /* any-hit rays traced since the last reset */
  int64_t nonfinite_dropped; /* contributions dropped because they were not finite */
  int64_t samples;           /* path samples started */
  double ms_extend;          /* summed kernel time of the traversal kernel: closest hits of a
                                bounce and shadow rays of the bounce before (profiling on) */
  int64_t launches_extend;   /* its launch count (profiling on) */
  double ms_total;           /* summed time of all sampling passes (profiling on) */
  int64_t node_visits;       /* BVH node fetches of closest-hit rays (counting on) */
  int64_t tri_tests;         /* triangle tests of closest-hit rays (counting on) */
  int64_t shadow_node_visits;/* BVH node fetches of shadow rays (counting on; tail kernel apart) */
  int64_t shadow_tri_tests;  /* triangle tests of shadow rays (counting on; tail kernel apart) */
  int64_t cache_queries;     /* paths that ended in the radiance cache */
  int64_t cache_records;     /* training records produced by the frames' training paths */
  int64_t cache_adam_steps;  /* Adam steps applied since the cache was configured or given weights */
  double ms_cache_query;     /* summed time of the cache-query kernel (profiling on) */
  double ms_cache_train;     /* summed time of training: targets and Adam steps (profiling on) */
  int64_t tail_extension_rays; /* closest-hit rays of the tail kernel (included in extension_rays) */
  int64_t tail_node_visits;  /* their node fetches (counting on; not in node_visits) */
  int64_t tail_tri_tests;    /* their triangle tests (counting on; not in tri_tests) */
  double ms_tail;            /* summed time of the tail kernel (profiling on) */
  int64_t launches_tail;     /* its launch count (profiling on) */
  int64_t tail_shadow_rays;  /* shadow rays of the tail kernel (included in shadow_rays) */
  int64_t tail_shadow_node_visits; /* their node fetches (counting on; not in shadow_node_visits) */
  int64_t tail_shadow_tri_tests;   /* their triangle tests (counting on; not in shadow_tri_tests) */
  double ms_display;         /* summed time of the display kernel (profiling on) */
  int64_t launches_display;  /* its launch count (profiling on) */
  int64_t instances_entered; /* two-level scenes: instances whose mesh walk started, closest-hit and
                                shadow walks of the traversal kernel (counting on; tail kernel apart) */
  int64_t tail_instances_entered; /* the same for the tail kernel's walks (counting on) */
  double ms_cache_forward;   /* summed kernel time of pt_nrc_forward calls (profiling on) */
  int64_t cache_forward_queries; /* queries answered by those calls (profiling on) */
} pt_stats;

/* Create a scene bound to HIP device `hip_device` and stream `hip_stream`
 * (a hipStream_t, or NULL for the default stream).  Allocates nothing on the
 * device yet.  Errors: INVALID_ARG (out == NULL), DEVICE. */
pt_status pt_scene_create(int32_t hip_device, void* hip_stream, pt_scene** out);

/* Release the scene and its device memory.  NULL-safe. */
void pt_scene_destroy(pt_scene* scene);

/* Build the acceleration structure on the CPU (Sec. 5.1.1: boxes grouped so
 * that every child lies inside its parent) and upload it.  With
 * n_instances == 0 the meshes are concatenated into one world-space mesh
 * and primitive ids number the concatenation; otherwise each instance
 * places meshes[mesh] and primitive ids are per mesh.
 * Errors: INVALID_ARG (NULL pointers, counts <= 0, indices out of range,
 * non-finite vertices or transforms, mesh index out of range), OUT_OF_MEMORY, DEVICE. */
pt_status pt_build_bvh(pt_scene* scene, const pt_mesh* meshes, int32_t n_meshes,
                       const pt_instance* instances, int32_t n_instances);

/* The same acceleration structure built on the GPU instead (the paper times
 * its CPU set-up as its own stage, Sec. 5.1.1, Table 1): triangles sorted by
 * 30-bit Morton codes of their centroids, a binary tree over them (by
 * default locally-ordered clustering: neighbours in the sorted order whose
 * merged box has the least surface area merge, round by round; else a linear
 * BVH, see pt_set_gpu_bvh_builder), collapsed top-down to the same 128-byte
 * BVH4 nodes and 48-byte triangle records.  Arguments,
 * primitive numbering and errors as pt_build_bvh; the tree differs, the
 * closest hits do not (a hit is defined by the triangle test alone).  With
 * instances each mesh's BVH is built on the GPU and the top level over the
 * instance boxes on the CPU.  Error: DEVICE if a device step fails (the scene
 * then has no BVH).  pt_scene_bvh_info reports its build time. */
pt_status pt_build_bvh_gpu(pt_scene* scene, const pt_mesh* meshes, int32_t n_meshes,
                           const pt_instance* instances, int32_t n_instances);

/* Builders of pt_build_bvh_gpu. */
typedef enum {
  PT_GPU_BVH_PLOC = 0, /* locally-ordered clustering (Meister & Bittner 2018): the default */
  PT_GPU_BVH_LBVH = 1  /* linear BVH (Karras 2012): binary radix tree over the sorted codes */
} pt_gpu_bvh_builder;

/* Choose the builder of the scene's later pt_build_bvh_gpu calls (an
 * acceleration-structure choice only: every closest hit is the same).
 * Error: INVALID_ARG (builder not one of pt_gpu_bvh_builder). */
pt_status pt_set_gpu_bvh_builder(pt_scene* scene, int32_t builder);

/* Upload the OpenPBR materials (Sec. 4).  base_diffuse_roughness > 0 gives
 * the energy-preserving Oren-Nayar diffuse (EON); specular_weight modulates
 * the dielectric IOR (F0(eta') = specular_weight F0(eta)) and scales the
 * metal Fresnel.  thin_film_weight > 0 puts a thin film (thickness in
 * micrometres, thin_film_ior >= 1) on the dielectric interface: its
 * reflectance is the interference (Airy) sum of the film, evaluated at 650,
 * 550 and 450 nm for red, green and blue, mixed with the plain Fresnel by
 * the weight; metals ignore the film.  fuzz_weight > 0 adds a sheen lobe
 * on top of everything else (Charlie distribution, alpha = fuzz_roughness^2
 * clamped below at 0.01, tinted by fuzz_color), which attenuates the layers
 * below by its directional albedo; the albedo table is computed here, once
 * per distinct alpha.  subsurface_weight > 0 mixes subsurface_color into the
 * albedo of the dielectric base's diffuse lobe (the subsurface's local limit,
 * see pt_openpbr_material).  Errors: INVALID_ARG (n <= 0, negative or
 * non-finite parameters, IOR <= 0, thin_film_ior < 1, weights,
 * fuzz_roughness or base_diffuse_roughness outside [0,1]), UNSUPPORTED (coat
 * or fuzz together with transmission). */
pt_status pt_upload_materials(pt_scene* scene, const pt_openpbr_material* materials, int32_t n);

/* Set the environment: an equirectangular RGB32F image [h][w][3] (y up,
 * theta = acos(d_y), phi = atan2(d_x, -d_z), column = (phi/2pi + 1/2) w,
 * row = theta/pi h), or NULL for none.  Builds its sampling tables.
 * Errors: INVALID_ARG (w or h <= 0, negative or non-finite texels). */
pt_status pt_set_environment(pt_scene* scene, const float* rgb32f, int32_t w, int32_t h);

/* Render: reset the FP64 per-pixel sums, accumulate samples [0, spp) of
 * every pixel with paths of at most max_depth scattering events, and write
 * the per-pixel mean to out_rgb32f (device, [height][width][3] float).
 * seed keys the Philox stream.  Errors: INVALID_ARG (camera, spp <= 0,
 * max_depth outside [0, 64], out == NULL), STATE (no BVH or materials,
 * a material id >= the material count), DEVICE. */
pt_status pt_render(pt_scene* scene, const pt_camera* camera, int32_t spp, int32_t max_depth,
                    uint64_t seed, float* out_rgb32f);

/* Progressive rendering (Sec. 5.1.4 shows the running mean after every
 * sampling iteration): add samples [first_sample, first_sample + n_samples)
 * to the FP64 sums.  The sums are reset when the camera's width or height
 * changes or by pt_reset_accumulation.  Splitting a range into several calls
 * gives bit-identical sums. */
pt_status pt_accumulate(pt_scene* scene, const pt_camera* camera, int32_t first_sample,
                        int32_t n_samples, int32_t max_depth, uint64_t seed);
pt_status pt_reset_accumulation(pt_scene* scene);

/* Write sum / samples_accumulated to out_rgb32f (device, [h][w][3] float),
 * and optionally copy the raw FP64 sums to out_sum_f64 (device, [h][w][3]
 * double, or NULL).  Errors: STATE if nothing was accumulated. */
pt_status pt_resolve(pt_scene* scene, float* out_rgb32f, double* out_sum_f64);

/* Replace the FP64 sums and their sample count (resuming a progressive
 * render from sums saved with pt_resolve's out_sum_f64): sum (device,
 * [height][width][3] double, copied) holds the sums of `samples` samples per
 * pixel.  A later pt_accumulate with a camera of the same size adds to them.
 * Errors: INVALID_ARG (sum NULL, width, height or samples <= 0), DEVICE. */
pt_status pt_set_accumulation(pt_scene* scene, const double* sum, int32_t width, int32_t height, int64_t samples);

/* Display image of the running mean (Sec. 5.1.4: the mean of the samples
 * accumulated so far is tone mapped with Khronos PBR Neutral and shown after
 * every sampling iteration).  Per pixel, in FP64: c = (sum / samples) *
 * exposure; PBR Neutral (the smallest channel x sets an offset x - 6.25 x^2
 * for x < 0.08, else 0.04, subtracted from every channel; a peak p at or
 * above 0.76 is compressed to q = 1 - 0.0576 / (p - 0.56), the colour scaled
 * by q / p and mixed towards grey q by 1 - 1 / (0.15 (p - q) + 1)); the sRGB
 * transfer function on [0, 1]; code floor(255 e + 1/2).  out_rgba8 (device,
 * [height][width] uint32, bytes R, G, B, A = 255 in memory order) and
 * out_encoded (device, [height][width][3] float, the sRGB values before
 * quantisation) are caller-owned; either may be NULL, not both.  Reads the
 * sums left by pt_render / pt_accumulate without changing them, so calling
 * it after every pt_accumulate gives the progressive display.
 * Errors: INVALID_ARG (both outputs NULL, exposure negative or not finite),
 * STATE (nothing accumulated), DEVICE. */
pt_status pt_display(pt_scene* scene, double exposure, uint32_t* out_rgba8, float* out_encoded);

/* Per-path output for parity checks: render samples [first_sample,
 * first_sample + spp) of the pixels in the crop (x0, y0, w, h) of the
 * camera's image and write each path's radiance to per_sample_rgb (device,
 * [h][w][spp][3] float) and its event signature to signature (device,
 * [h][w][spp] uint64, FNV-1a 64 over the path's events).  Uses the same
 * kernels as pt_render with the signature bookkeeping switched on. */
pt_status pt_render_debug(pt_scene* scene, const pt_camera* camera, int32_t x0, int32_t y0,
                          int32_t w, int32_t h, int32_t first_sample, int32_t spp,
                          int32_t max_depth, uint64_t seed, float* per_sample_rgb,
                          uint64_t* signature);

/* Closest hit of n rays (device, [n][8] float: ox, oy, oz, tmin, dx, dy, dz,
 * tmax) written to hits (device, [n][6] uint32: t bits, instance, primitive,
 * b1 bits, b2 bits, 1 if hit; a miss is +inf, 0xFFFFFFFF, 0xFFFFFFFF, 0, 0, 0).
 * brute_force != 0 tests every triangle instead of walking the BVH.  Ties
 * in t resolve to the smallest (instance, primitive). */
pt_status pt_trace_closest(pt_scene* scene, const float* rays, int64_t n, uint32_t* hits,
                           int32_t brute_force);

/* pt_trace_closest for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels, results bit-identical to pt_trace_closest,
 * but the traversal stack spill and the launch's counters live in a static
 * device array of the library (32 MiB, one copy per GPU, held until the
 * process ends) instead of scene buffers.  The call allocates nothing; the
 * caller passes rays and hits as for pt_trace_closest.  The grid of the BVH
 * walk shrinks until every lane's spill area fits the array.  Every call on
 * a GPU shares that GPU's array: calls that overlap on one GPU (several
 * host threads, or scenes on different streams of the same device) race
 * and must not be issued concurrently.  It adds nothing to pt_get_stats.
 * Errors: as pt_trace_closest; UNSUPPORTED if one workgroup's spill area of
 * this BVH's depth exceeds the array (a hierarchy far deeper than any
 * binned-SAH build of 2^31 triangles); DEVICE on a traversal stack overflow
 * (hits of that call may then be wrong). */
pt_status pt_trace_closest_noalloc(pt_scene* scene, const float* rays, int64_t n, uint32_t* hits,
                                   int32_t brute_force);

/* Statistics since the last pt_reset_stats. */
pt_status pt_get_stats(pt_scene* scene, pt_stats* out);
pt_status pt_reset_stats(pt_scene* scene);

/* Kernel timing with HIP events on the scene's stream (0 off, 1 on), and
 * node-visit / triangle-test counting (0 off, 1 on; uses a counting variant
 * of the traversal kernels). */
pt_status pt_set_profiling(pt_scene* scene, int32_t timing, int32_t counting);

/* ---- radiance cache ----
 * The paper names neural radiance caching as the way to need fewer samples
 * (Sec. 6.1, future work).  The cache here is a 64 -> 5 x 64 (ReLU) -> 3
 * network without biases over a fixed 64-feature encoding of 12 vertex
 * inputs (position in the scene box, outgoing direction and shading normal
 * as spherical pairs, specular roughness, diffuse albedo, specular
 * luminance), bfloat16 operands with FP32 sums, trained online with Adam
 * on the relative L2 loss (y - t)^2 / (y^2 + 0.01) (denominator held
 * constant).  Weights: W0..W4 (64 x 64) then W5 (3 x 64), row-major
 * [out][in], 20,672 floats.
 *
 * With the cache configured, pt_render / pt_accumulate run every sample
 * pass as one frame: the pass renders with the cache (once it has weights:
 * set by pt_nrc_set_weights or learnt in an earlier frame), paths that reach
 * vertex query_bounce below max_depth add beta * max(cache, 0) there and
 * stop; then train_paths training paths (plain paths, sample index
 * 2^31 + frame, pixels (k * floor(WH / train_paths) + o_frame) mod WH)
 * record (inputs, (L_end - L_k) / beta_k) at their vertices, and
 * steps_per_frame Adam steps run on batches of batch_size records drawn
 * with replacement by Philox (see pt_nrc_train).  A frame with no record
 * changes no weight and counts no step.  The frames of one call overlap on
 * the device (a frame's training beside the next frame's first bounces,
 * whose cache queries wait for it); images, weights and step counts are
 * bitwise those of one call per frame. */
typedef struct pt_radiance_cache_config {
  int32_t query_bounce;    /* vertex at which sampling paths end in the cache, >= 0 (2 by default) */
  int32_t train_paths;     /* training paths per frame, [1, 2^24] (65536) */
  int32_t batch_size;      /* records per Adam step, [1, 2^22] (16384) */
  int32_t steps_per_frame; /* Adam steps per frame, [0, 64] (4) */
  float learning_rate;     /* > 0 (1e-3) */
  float beta1, beta2;      /* in [0, 1) (0.9, 0.99) */
  float epsilon;           /* > 0 (1e-8) */
  uint64_t init_seed;      /* Philox key of the He-uniform initial weights */
  float ema_decay;         /* [0, 1): after each Adam step t the moving average e = ema_decay e +
                              (1 - ema_decay) w (e starts at 0) is updated and the cache queries use
                              e / (1 - ema_decay^t); 0 uses the weights themselves (0) */
  int32_t train_end_bounce; /* self-training, >= -1: once the cache has weights, a training path
                              that reaches this vertex below max_depth ends there in the cache (no
                              record at that vertex; beta * cache(x) joins its radiance before the
                              targets of its earlier vertices are formed); -1: plain training paths
                              to max_depth (-1) */
  float spread_c;          /* >= 0: adaptive termination of the cited method: a sampling path ends in the
                              cache at the first vertex b >= 1 where (sum over its non-delta bounces of
                              sqrt(t_i^2 / (pdf_i |cos theta_i|)))^2 > spread_c * t_0^2 / (4 pi
                              |cos theta_0|) (t: hit distance, pdf: solid-angle pdf of the bounce
                              into that vertex, theta: angle to the geometric normal there), and at
                              query_bounce at the latest; 0: always at query_bounce (0) */
  int32_t factorize;       /* 0 or 1: the network predicts radiance divided, per channel, by
                              (diffuse albedo + specular albedo) of the vertex (inputs 8..10 and
                              11); queries multiply by that factor, targets are divided by it and
                              dropped where it is zero (0) */
} pt_radiance_cache_config;

/* Configure (cfg != NULL) or switch off (cfg == NULL) the cache.  Weights
 * start He-uniform: weight k of layer l is (2u - 1) sqrt(6/64), u the
 * Philox uniform at counter (k, l, 0x4E5243, 0) under init_seed; Adam
 * moments, the moving average and the step count start at zero; rendering does not use the cache
 * until it has been trained or given weights.  Errors: INVALID_ARG for a
 * field out of range, DEVICE. */
pt_status pt_set_radiance_cache(pt_scene* scene, const pt_radiance_cache_config* cfg);

/* Replace the weights (device, 20,672 floats, copied), reset the Adam state
 * and let rendering use the cache.  Errors: STATE if not configured,
 * INVALID_ARG if weights == NULL or n != 20672. */
pt_status pt_nrc_set_weights(pt_scene* scene, const float* weights, int64_t n);

/* Copy the FP32 master weights and the Adam moments (device, 20,672 floats
 * each; any pointer may be NULL) and the number of Adam steps taken. */
pt_status pt_nrc_get_weights(pt_scene* scene, float* weights, float* adam_m, float* adam_v, int64_t* step);

/* The inference weights the cache queries use (device, 20,672 floats): the
 * bias-corrected moving average after Adam steps with ema_decay > 0, else
 * the weights; equal to the weights before the first step and after
 * pt_nrc_set_weights. */
pt_status pt_nrc_get_inference_weights(pt_scene* scene, float* weights);

/* Cache outputs of n inputs under the inference weights: inputs (device,
 * [n][12] float) -> outputs (device, [n][3] float, unclamped).  The same
 * kernel code answers the queries of the sampling passes. */
pt_status pt_nrc_forward(pt_scene* scene, const float* inputs, int64_t n, float* outputs);

/* Gradient of the mean loss over n samples (device inputs [n][12], targets
 * [n][3]) with respect to the 20,672 weights, written to grad (device);
 * loss (host, may be NULL) receives the mean loss.  No weights change.
 * The sums over samples run in a fixed order, so repeated calls agree bit
 * for bit.  Errors: INVALID_ARG for n outside [1, 2^22]. */
pt_status pt_nrc_gradient(pt_scene* scene, const float* inputs, const float* targets, int32_t n, float* grad,
                          double* loss);

/* One frame's training on n given records (device inputs [n][12], targets
 * [n][3]): steps_per_frame Adam steps; the batch of step s has batch_size
 * samples, sample j taking record floor(m * n / 2^24) with m the top 24 bits
 * of Philox word s mod 4 at counter (j, 2^31 + frame, 0x4E5253, s / 4) under
 * seed.  mean_loss (host, may be NULL) receives the mean of the steps'
 * losses (before each update).  Used by the frame loop on the records of
 * the frame's training paths. */
pt_status pt_nrc_train(pt_scene* scene, const float* inputs, const float* targets, int32_t n, int32_t frame,
                       uint64_t seed, double* mean_loss);

/* Trace the training paths of a frame and return their records, path by path
 * in vertex order: inputs (device, [capacity][12]), targets (device,
 * [capacity][3]), path_offsets (device, [train_paths] uint32, first record of
 * each path, or NULL); *n_records receives the total, of which
 * min(total, capacity) are written.  No weights change. */
pt_status pt_nrc_training_records(pt_scene* scene, const pt_camera* camera, int32_t frame, int32_t max_depth,
                                  uint64_t seed, float* inputs, float* targets, uint32_t* path_offsets,
                                  int64_t capacity, int64_t* n_records);

/* Tail hand-off of the sampling passes.  A pass runs the wavefront kernels
 * (one launch per stage per bounce) while many paths are alive; from bounce
 * min_bounce on, once at most max_fraction of the pass's paths are still
 * alive, one persistent kernel runs all remaining vertices of every path
 * (closest hit, shading, shadow ray, next ray) without a kernel boundary
 * per bounce.  The decision reads one counter back per pass.  Results are
 * identical either way (same arithmetic, same random numbers).  Defaults:
 * min_bounce 2, max_fraction 0.15; max_fraction 0 (or min_bounce > 64)
 * keeps the wavefront throughout.  Errors: INVALID_ARG for min_bounce < 0
 * or max_fraction outside [0, 1]. */
pt_status pt_set_tail(pt_scene* scene, int32_t min_bounce, double max_fraction);

/* ---- host-only BVH access (no device needed) ---- */
typedef struct pt_bvh_host pt_bvh_host;
typedef struct pt_bvh_info {
  int64_t n_nodes;        /* 128-byte BVH4 nodes */
  int64_t n_tris;         /* 48-byte triangle records in leaf order */
  int32_t depth;          /* nodes on the longest root-to-leaf path */
  int32_t max_leaf_tris;
  double sah_cost;
  double build_ms;
  int32_t stack_capacity; /* traversal stack entries per lane the GPU walk is given: three per
                             inner level plus one top-level leaf's instances (3 * depth +
                             max leaf size), which bounds every walk of this hierarchy */
} pt_bvh_info;
/* The scene's mesh-level BVH (either builder): node and triangle counts,
 * depth, largest leaf, SAH cost (host builds; 0 for device builds),
 * build_ms from the triangle soup in host memory to the BVH in the builder's
 * memory (device builds: soup upload included; two-level: summed over the
 * meshes), and the traversal stack capacity.  Errors: STATE without a BVH. */
pt_status pt_scene_bvh_info(pt_scene* scene, pt_bvh_info* info);
/* Copy the scene's mesh-level BVH to host memory: nodes (n_nodes * 128
 * bytes, root at 0; two-level scenes: the meshes' trees concatenated) and
 * triangles (n_tris * 48 bytes, leaf order); either may be NULL. */
pt_status pt_scene_copy_bvh(pt_scene* scene, void* nodes, void* tris);

/* Build the BVH4 of one mesh on the host (the same builder pt_build_bvh uses). */
pt_status pt_bvh_host_build(const pt_mesh* mesh, pt_bvh_host** out);
/* Build the two-level hierarchy of an instanced scene on the host (the same
 * code pt_build_bvh runs for n_instances > 0); nodes / triangles then refer
 * to the concatenated per-mesh BVHs. */
pt_status pt_bvh_host_build_instanced(const pt_mesh* meshes, int32_t n_meshes, const pt_instance* instances,
                                      int32_t n_instances, pt_bvh_host** out);
pt_status pt_bvh_host_info(const pt_bvh_host* bvh, pt_bvh_info* info);
/* Copy nodes (n_nodes * 128 bytes) and triangles (n_tris * 48 bytes) to host memory. */
pt_status pt_bvh_host_copy(const pt_bvh_host* bvh, void* nodes, void* tris);
/* Closest hit on the host through the BVH4 (same traversal code as the GPU,
 * compiled for the CPU).  rays/hits as for pt_trace_closest, host memory. */
pt_status pt_bvh_host_trace(const pt_bvh_host* bvh, const float* rays, int64_t n, uint32_t* hits);
/* The same walk with a stack of `stack_capacity` entries per ray (<= 0: the
 * capacity pt_bvh_info reports; at most 512), for checking the stack bound
 * on the CPU.  *high_water (nullable) receives the deepest stack any ray
 * used.  A push beyond the capacity is dropped as on the GPU, and the call
 * then fails with PT_ERR_DEVICE ("traversal stack overflow"); hits of the
 * rays traced so far are still written. */
pt_status pt_bvh_host_trace_stack(const pt_bvh_host* bvh, const float* rays, int64_t n, uint32_t* hits,
                                  int32_t stack_capacity, int32_t* high_water);
void pt_bvh_host_destroy(pt_bvh_host* bvh);

/* Thread-local message of the last failed call on this thread ("" if none). */
const char* pt_last_error(void);

/* Library version string. */
const char* pt_version(void);

#ifdef __cplusplus
}
#endif
#endif

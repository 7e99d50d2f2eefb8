/*
 * svraster.h -- C ABI of the MI355X (gfx950) sparse-voxel rasterizer.
 *
 * The library renders octree-leaf voxels ("Sparse Voxels Rasterization",
 * Sun et al., CVPR 2025, arXiv 2412.04459) and back-propagates into their
 * parameters.  One frame is four calls, in this order, on one stream:
 *
 *   svr_preprocess  project voxels to screen tiles (16x16 by default), pre-process the
 *                   per-view voxel records and duplicate voxels per tile and
 *                   ray-sign pattern                   (Sec. 3.1.2, Supp. B.1)
 *   svr_sort        sort the duplicated list by tile and direction-dependent
 *                   Morton order                       (Sec. 3.1.2, Supp. B.2)
 *   svr_render_fwd  front-to-back alpha compositing of every pixel
 *                   (Sec. 3.1 eq. alpha_blend, Sec. 3.1.1 eq. vox_alpha and
 *                   eq. vox_color, Sec. 3.1.2 "Rendering pixels")
 *   svr_render_bwd  the adjoint of svr_render_fwd into corner raw densities
 *                   and SH coefficients (Supp. A.2, gradient of alpha)
 *
 * Conventions shared by every call:
 *   - All array pointers inside svr_scene, and the rgba / gradient pointers,
 *     are DEVICE pointers, caller-owned, contiguous, little-endian, fp32 unless
 *     noted.  svr_camera arrays and svr_opts are HOST memory, read during the
 *     call only.
 *   - `ws` is a caller-allocated device workspace of at least
 *     svr_workspace_bytes() bytes.  The library allocates nothing.  The
 *     workspace carries the state from one call to the next of the same frame
 *     (sorted list, per-pixel saved state); it must not be modified or reused
 *     for another frame between svr_preprocess and the last svr_render_bwd of
 *     that frame.  Distinct workspaces may be used concurrently.
 *   - Every call enqueues its work asynchronously on `stream` (a hipStream_t;
 *     NULL is the default stream) and returns a status code.  The only
 *     host-visible synchronisation is in svr_preprocess when `n_entries_out`
 *     is not NULL (one 8-byte read-back).
 *   - No C++ exception crosses the ABI.  svr_last_error() describes the last
 *     failing call of the calling thread.
 *   - Camera model: OpenCV pinhole (x right, y down, z forward), world-to-camera
 *     [R | t] row-major; the ray of pixel (u, v) leaves the camera centre
 *     -R^T t along normalize(R^T ((u+0.5-cx)/fx, (v+0.5-cy)/fy, 1)).
 */
#ifndef SVRASTER_H
#define SVRASTER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------- */
#define SVR_OK 0
#define SVR_E_INVALID (-1)   /* bad argument: null pointer, limit exceeded, bad enum */
#define SVR_E_CAPACITY (-2)  /* duplicated list exceeds opts.entry_capacity          */
#define SVR_E_HIP (-3)       /* a HIP runtime call failed                            */
#define SVR_E_WORKSPACE (-4) /* ws_bytes smaller than svr_workspace_bytes()          */
#define SVR_E_DEVICE (-5)    /* a kernel reported an internal failure (see text)     */

/* ---- enums and limits ---------------------------------------------------- */
#define SVR_ACT_EXPLIN 0     /* Sec. 3.1.1 eq. explin                                */
#define SVR_ACT_SOFTPLUS 1   /* softplus with beta = 1                               */
#define SVR_MAX_CAMERAS 32   /* cameras per call                                     */
#define SVR_MAX_LEVELS 16    /* octree levels (Supp. A.1)                            */
#define SVR_MAX_VOXELS (1 << 29) /* voxel ids are 29 bits in a value (Supp. B.1)     */
#define SVR_MAX_K 8          /* samples per ray-voxel segment                        */
#define SVR_TILE 16          /* default tile edge in pixels                          */

/* Scene (Sec. 3.1.1): leaf voxels in arbitrary order, corner grid points
 * shared between voxels, per-voxel SH.  All pointers are device pointers.   */
typedef struct svr_scene {
  int64_t n_voxels;        /* N, 0 <= N < 2^29                                         */
  int64_t n_grid;          /* M, number of corner grid points                          */
  const float* center;     /* [3][N] voxel centres, SoA (x row, y row, z row)          */
  const float* size;       /* [N]    voxel edge lengths                                */
  const uint64_t* octpath; /* [N]    octree path: the octant (4x+2y+z) of level l sits
                              at bits 3(16-l)..3(16-l)+2; unused low triplets zero
                              (Supp. A.1 listing for the index <-> path conversion)   */
  const int32_t* vox_grid; /* [N][8] grid point of corner c = 4dx + 2dy + dz          */
  const float* grid_raw;   /* [M]    raw (pre-activation) densities                   */
  const float* sh;         /* [N][(D+1)^2][3] SH coefficients, basis index l*l+l+m    */
  int32_t sh_degree;       /* D in 0..3                                                */
  int32_t max_level;       /* deepest level present, 1..16                             */
  const int32_t* grid_adj_off; /* [M+1] optional (NULL: atomics): corner adjacency of   */
  const int32_t* grid_adj;     /* [8N]  the grid points, see svr_build_grid_adjacency   */
  const uint32_t* order_rank;  /* [N][8] optional (NULL: keys from octpath): order ranks
                                  of the (voxel, sign) pairs, see svr_build_order_ranks */
} svr_scene;

/* Pinhole camera (host memory). */
typedef struct svr_camera {
  int32_t width, height;   /* pixels, 1..16384                                         */
  float fx, fy, cx, cy;    /* intrinsics in pixels                                     */
  float w2c[12];           /* world-to-camera [R | t], row-major 3x4                   */
} svr_camera;

/* Options (host memory). */
typedef struct svr_opts {
  int32_t K;               /* samples per ray-voxel segment, 1..8 (eq. vox_alpha)      */
  float t_stop;            /* early termination threshold on transmittance (h_T)      */
  int32_t activation;      /* SVR_ACT_EXPLIN or SVR_ACT_SOFTPLUS                       */
  int32_t tile;            /* tile edge in pixels: 8, 16 or 32 (0 means 16)            */
  int64_t entry_capacity;  /* capacity of the duplicated (tile, voxel, sign) list, < 2^30 */
  int32_t persistent;      /* 0: one render workgroup per tile; n > 0: n workgroups take
                              tiles (heaviest first) from a counter until all are done */
  int32_t accumulate;      /* svr_render_bwd: 0 overwrites grad_grid / grad_sh, 1 adds
                              into them (several camera groups, one gradient)          */
} svr_opts;

/* Bytes of workspace one frame of `n_cams` cameras needs with
 * opts->entry_capacity entries.  Returns 0 on invalid arguments. */
size_t svr_workspace_bytes(const svr_scene* scene, const svr_camera* cams, int n_cams,
                           const svr_opts* opts);

/* The same workspace split by purpose, in bytes (alignment padding included),
 * written to parts[0 .. min(n_parts, SVR_WS_PARTS) - 1]:
 *   [0] header, tile masks, tile summed-area table, tile ranges, render order,
 *       per-tile entry counts (counting sort) and the backward chunk list of
 *       heavy tiles
 *   [1] per (voxel, camera): count, tile rectangle and render record
 *   [2] scan partial sums
 *   [3] sort keys and values, both buffers of the double-buffered sort
 *   [4] radix-sort digit histograms and look-back status
 *   [5] per-pixel saved state of the forward (final optical depth, last entry,
 *       and the checkpoints at chunk boundaries of heavy tiles)
 *   [6] gradient scratch (per-voxel corner gradients, per (voxel, camera) colour)
 * The parts sum to svr_workspace_bytes().  Returns SVR_OK or SVR_E_INVALID. */
#define SVR_WS_PARTS 7
int svr_workspace_parts(const svr_scene* scene, const svr_camera* cams, int n_cams,
                        const svr_opts* opts, size_t* parts, int n_parts);

/* Projection and pre-processing (Sec. 3.1.2 "Projection to image space",
 * "Pre-processing voxels"; duplication per tile and ray-sign pattern,
 * Supp. B.1).
 * For every camera and voxel: project the 8 corners and assign the voxel to
 * every tile overlapped by the box of the projections (voxels outside the
 * view frustum are culled; one with a corner closer than 1e-4 to the camera
 * plane is assigned every tile); gather its 8 corner densities and evaluate
 * its SH colour for the direction from the camera centre to the voxel centre;
 * then emit one (key, value) entry per (tile, ray-sign pattern present among
 * that tile's pixels).  key = tile << (3 max_level + 3) | order << 3 | s with
 * order the top 3 max_level bits of the direction-dependent Morton code
 * (Supp. B.2), value = s << 29 | voxel id.
 *   n_entries_out  host pointer receiving the entry count E; the call then
 *                  reads E back (one synchronisation) and returns
 *                  SVR_E_CAPACITY, with *n_entries_out = E, when E exceeds
 *                  opts->entry_capacity (nothing is emitted then).  NULL: no
 *                  synchronisation; overflow is reported later by
 *                  svr_check_overflow() and the list is truncated.
 * Errors: SVR_E_INVALID, SVR_E_WORKSPACE, SVR_E_CAPACITY, SVR_E_HIP.        */
int svr_preprocess(const svr_scene* scene, const svr_camera* cams, int n_cams,
                   const svr_opts* opts, void* ws, size_t ws_bytes, int64_t* n_entries_out,
                   void* stream);

/* Sort the duplicated list by key (ascending; keys are unique whenever
 * max_level <= 15, so the order is fully determined) (Sec. 3.1.2 "Sorting
 * voxels"): the entries are first bucketed by tile, then every tile's
 * [start, end) range is sorted by the key's low bits (the
 * direction-dependent order).  The bucketing is a counting sort (per-tile
 * counts, their scan, one placement pass) when the frame has at most 32768
 * tiles and the keys are unique within a tile (order ranks, or max_level <=
 * 15), else an LSD radix sort over the key's tile bits; both give the same
 * list.  Must follow svr_preprocess on the same workspace (which clears the
 * per-tile counts); tile counts that disagree with the entry count leave
 * every range empty and make svr_check_overflow return SVR_E_DEVICE.
 * `n_entries_hint` is E when known (it sizes the launches) or -1 to size
 * them by capacity; the device-side count is authoritative either way.
 * Errors: SVR_E_INVALID, SVR_E_WORKSPACE, SVR_E_HIP.                         */
int svr_sort(const svr_scene* scene, const svr_camera* cams, int n_cams, const svr_opts* opts,
             void* ws, size_t ws_bytes, int64_t n_entries_hint, void* stream);

/* Optional extra outputs and inputs of the render calls.  Every pointer is
 * caller-owned device memory or NULL (feature off).
 * Per-voxel training statistics (Sec. 3.2.2 "Adaptive Pruning and
 * Subdivision"), arrays of n_voxels floats that the calls accumulate into
 * across cameras and calls (maximum / sum), so the caller zeroes them at the
 * start of a statistics window:
 *   max_weight   svr_render_fwd: max over composited hits of the blending
 *                weight T_i alpha_i (the pruning test)
 *   priority     svr_render_bwd: sum over composited hits of
 *                |alpha_i dL/dalpha_i| (eq. priority, the subdivision order;
 *                L is the rgba loss)
 * Depth and normal images (Sec. 3.1.1 "Voxel normal", "Voxel depth";
 * Supp. details of voxel normal and depth), overwritten:
 *   depth        svr_render_fwd: [P] D = sum_i T_i d_i, d_i the voxel's K
 *                samples composited with their own alphas at their ray
 *                distances t_k
 *   normal       svr_render_fwd: [P][3] N = sum_i T_i alpha_i n_i, n_i the
 *                normalised gradient of the voxel's trilinear raw density at
 *                its centre (as printed: it points to increasing density)
 *   grad_depth   svr_render_bwd: [P] dL/dD (NULL: 0)
 *   grad_normal  svr_render_bwd: [P][3] dL/dN (NULL: 0)
 * A backward with grad_depth or grad_normal needs the frame's forward to have
 * produced depth and normal (it saves their partial sums for the backward).  */
typedef struct svr_extra {
  float* max_weight;
  float* priority;
  float* depth;
  float* normal;
  const float* grad_depth;
  const float* grad_normal;
} svr_extra;

/* Render (Sec. 3.1 eq. alpha_blend; Sec. 3.1.1 eq. vox_alpha, eq. explin,
 * eq. vox_color; Supp. A.2 eq. K_samp_pts, eq. interp; Sec. 3.1.2 "Rendering
 * pixels").  Each pixel walks its tile's sorted list; entries of another
 * sign pattern and voxels its ray misses (ray-box slab test, entry distance
 * > 0) are skipped; a voxel is composited iff the transmittance before it is
 * >= t_stop.  Output rgba: [sum_c H_c W_c][4], cameras in order, row-major
 * pixels; premultiplied RGB and A = 1 - T_final (no background).  `extra`
 * may be NULL; its max_weight, depth and normal are written here.
 * Errors: SVR_E_INVALID, SVR_E_WORKSPACE, SVR_E_HIP.  A failure a kernel
 * detects on the device is flagged in the workspace header and returned as
 * SVR_E_DEVICE by the next svr_check_overflow.                              */
int svr_render_fwd(const svr_scene* scene, const svr_camera* cams, int n_cams,
                   const svr_opts* opts, void* ws, size_t ws_bytes, float* rgba,
                   const svr_extra* extra, void* stream);

/* Adjoint of svr_render_fwd for L = sum <grad_rgba, rgba>.  The transmittance
 * is recomputed walking each pixel's list back to front from the saved final
 * optical depth (no per-sample state is stored).  Outputs are overwritten
 * (added into when opts->accumulate is 1):
 *   grad_grid  [M]                 dL/d grid_raw            (may be NULL)
 *   grad_sh    [N][(D+1)^2][3]     dL/d sh                  (may be NULL)
 * `extra` may be NULL; its grad_depth and grad_normal are read and its
 * priority is accumulated here.
 * Errors: SVR_E_INVALID, SVR_E_WORKSPACE, SVR_E_HIP.  A failure a kernel
 * detects on the device (a backward chunk list that would overflow) is
 * flagged in the workspace header and returned as SVR_E_DEVICE by the next
 * svr_check_overflow.                                                       */
int svr_render_bwd(const svr_scene* scene, const svr_camera* cams, int n_cams,
                   const svr_opts* opts, void* ws, size_t ws_bytes, const float* grad_rgba,
                   float* grad_grid, float* grad_sh, const svr_extra* extra,
                   void* stream);

/* After the frame (synchronises `stream`): *required_entries = E of the last
 * svr_preprocess on this workspace.  Returns SVR_E_CAPACITY if E exceeded
 * the capacity, SVR_E_DEVICE if a kernel flagged an internal failure. */
int svr_check_overflow(const svr_scene* scene, const svr_camera* cams, int n_cams,
                       const svr_opts* opts, void* ws, size_t ws_bytes,
                       int64_t* required_entries, void* stream);

/* Read back the sorted list of the frame (debug / parity): keys[E], values[E]
 * device pointers of capacity >= E.  Keys are tile << (3L + 3) | (top 3L path
 * bits XOR s * 0b001..001) << 3 | s, or tile << ceil(log2(8N)) | rank when the
 * scene carries order ranks; values are s << 29 | voxel id.  Asynchronous. */
int svr_copy_sorted(const svr_scene* scene, const svr_camera* cams, int n_cams,
                    const svr_opts* opts, void* ws, size_t ws_bytes, uint64_t* keys,
                    uint32_t* values, int64_t n, void* stream);

/* Stand-alone stable LSD radix sort of (key, value) pairs on bits [0, bits)
 * of the keys, the sort svr_sort runs (Supp. B.1 "GPU Radix sort").
 * keys/values: device [n], sorted in place.  keys_tmp/values_tmp: device [n]
 * scratch.  scratch: device, >= svr_radix_sort_scratch_bytes(n, bits).
 * Errors: SVR_E_INVALID, SVR_E_WORKSPACE, SVR_E_HIP.                         */
size_t svr_radix_sort_scratch_bytes(int64_t n, int bits);
int svr_radix_sort_pairs(uint64_t* keys, uint32_t* values, uint64_t* keys_tmp,
                         uint32_t* values_tmp, int64_t n, int bits, void* scratch,
                         size_t scratch_bytes, void* stream);

/* svr_radix_sort_pairs for callers that cannot allocate (code under stream
 * or graph capture, tight serving loops, hosts that forbid allocation): the
 * same sort with its second key/value buffer, counters, digit histograms
 * and look-back status in a device array the library holds, one copy per
 * GPU, SVR_STATIC_SORT_BYTES in size, kept until the process ends.  The
 * caller passes only the pairs.  Nothing is allocated: no hipMalloc, no
 * hipFree, no allocating library call.
 *   keys/values: device [n], sorted in place on bits [0, bits);
 *   n <= SVR_STATIC_SORT_MAX (larger n: SVR_E_INVALID, nothing launched);
 *   stream: a stream of the current device.
 * Every call on one GPU uses that GPU's array and leaves its contents from
 * the last call (the counters it needs zeroed are cleared by each call):
 * calls that overlap on one GPU (other streams, other host threads) race
 * and must be serialised by the caller.
 * Errors: SVR_E_INVALID, SVR_E_HIP.                                          */
#define SVR_STATIC_SORT_MAX (1 << 21)
#define SVR_STATIC_SORT_BYTES ((size_t)26223104)
int svr_radix_sort_pairs_static(uint64_t* keys, uint32_t* values, int64_t n, int bits,
                                void* stream);

/* Atomic throughput probe (measurement only): n_waves wave64 groups each
 * issue `iters` float atomic adds without return, in the pattern of the
 * render backward's gradient flush (Supp. A.2 gradients summed per wave,
 * then one atomic per value): per instruction, 8 lanes add 1.0 to the 32-byte
 * corner row and 3 lanes to the 12-byte colour row of a voxel drawn
 * uniformly from n_rows by a per-wave generator.  corner: device float
 * [n_rows][8]; colour: device float [n_rows][3]; both accumulated into (the
 * grand total grows by 11 n_waves iters).  1 <= n_rows < 2^32,
 * 1 <= n_waves <= 2^26, iters >= 0.
 * Errors: SVR_E_INVALID, SVR_E_HIP.                                          */
int svr_atomic_probe(float* corner, float* colour, int64_t n_rows, int64_t n_waves, int iters,
                     void* stream);

/* Frame statistics (diagnostics; synchronises `stream`), after svr_sort:
 *   counts[0]  entries E of the sorted list
 *   counts[1]  (pixel, entry) pairs with the pixel's sign pattern that the
 *              compositing loop of Sec. 3.1.2 walks (up to early termination)
 *   counts[2]  ray-box tests the render kernel executes after its culling
 *   counts[3]  composited ray-voxel hits
 *   counts[4]  (voxel, camera) pairs with at least one entry (in view)
 * Runs a counting variant of the render kernel; writes no image.
 * Errors: SVR_E_INVALID, SVR_E_WORKSPACE, SVR_E_HIP.                         */
int svr_render_stats(const svr_scene* scene, const svr_camera* cams, int n_cams,
                     const svr_opts* opts, void* ws, size_t ws_bytes, int64_t* counts,
                     void* stream);

/* Kernel timing (diagnostics, process-wide, not for concurrent use from
 * several threads): while enabled, every kernel launch of the library is
 * bracketed by HIP events on its own stream.  svr_timing_read waits for the
 * recorded events and returns, per kernel name (NUL-terminated, name_len bytes
 * per slot), the summed duration in milliseconds and the launch count since
 * the last read or enable, then clears the records.  At most 8192 launches
 * are recorded between reads.
 * Errors: SVR_E_INVALID, SVR_E_HIP.                                          */
int svr_timing_enable(int on);
int svr_timing_read(char* names, int name_len, double* total_ms, int64_t* launches, int max_n,
                    int* n_out);

/* Whole-frame hipGraph (the batched form: all cameras of the call in one
 * launch per stage, no host synchronisation).  svr_graph_capture records, on
 * `stream` (must not be the NULL stream), svr_preprocess (without read-back),
 * svr_sort (sized by capacity), svr_render_fwd into `rgba` and, when
 * grad_rgba is not NULL, svr_render_bwd into grad_grid / grad_sh (`extra` as
 * for those calls, NULL allowed); it returns
 * an executable graph in *graph_out.  Cameras and options are baked into the
 * graph; scene arrays, workspace and outputs are read and written through the
 * pointers given here at every replay.  svr_graph_launch replays it on a
 * stream; check capacity overflow with svr_check_overflow afterwards.
 * Kernel timing is suspended while capturing.  No device memory is allocated
 * (the graph objects are host-side).
 * Errors: SVR_E_INVALID, SVR_E_WORKSPACE, SVR_E_HIP.                         */
int svr_graph_capture(const svr_scene* scene, const svr_camera* cams, int n_cams,
                      const svr_opts* opts, void* ws, size_t ws_bytes, float* rgba,
                      const float* grad_rgba, float* grad_grid, float* grad_sh,
                      const svr_extra* extra, void* stream, void** graph_out);
int svr_graph_launch(void* graph, void* stream);
int svr_graph_destroy(void* graph);

/* Anti-aliasing (Sec. 3.1.2 "Anti-aliasing": render ss times larger, then
 * downsample with an anti-aliasing filter) and background colour (the
 * supplementary implementation details use the average frame colour).
 * svr_downsample: out[h_out][w_out][4] from in[h_in][w_in][4] (device, rgba as
 * svr_render_fwd writes it) by the separable tent of half-width
 * n_in / n_out per axis, centred at (i + 1/2) n_in / n_out - 1/2, weights
 * normalised over the in-image taps; then rgb += (1 - A) bg (bg: HOST
 * float[3], NULL for black).  svr_downsample_bwd: the adjoint, grad_in from
 * grad_out (overwritten).  Render at w_in x h_in with the intrinsics scaled by
 * w_in / w_out and h_in / h_out.
 * Errors: SVR_E_INVALID (sizes: 1 <= out <= in <= 65536, null pointers),
 * SVR_E_HIP.                                                                 */
int svr_downsample(const float* in, int w_in, int h_in, float* out, int w_out, int h_out,
                   const float* bg, void* stream);
int svr_downsample_bwd(const float* grad_out, int w_out, int h_out, float* grad_in, int w_in,
                       int h_in, const float* bg, void* stream);

/* Mesh extraction (Sec. 3.2.4 "Sparse-voxel TSDF Fusion and Marching Cubes").
 *
 * svr_tsdf_fuse: truncated signed distances at the grid points fused from
 * depth images.  For grid point p and camera i: when p projects (by
 * p_cam = R p + t of w2c as given) in front of the camera into pixel
 * (floor u, floor v) of the image (pixel centres at
 * +1/2) and that pixel holds depth D > 0 (distance along the unit ray;
 * D <= 0 marks no depth), sdf = D - |p - o_i|;
 * sdf >= -trunc adds min(sdf / trunc, 1) with weight 1.  tsdf[m] is the mean
 * of the added values (1 when none), weight[m] their count.
 * grid_pos: device float [3][n_grid] (x row, y row, z row); cams: host
 * [n_cams], any number >= 1 (one launch per group of consecutive cameras:
 * SVR_MAX_CAMERAS, or with order NULL as many as keep the images within
 * 96 MB; tsdf holds running sums in between); depth: device float, the
 * cameras'
 * [H][W] images concatenated in
 * camera order.  rgba: NULL (depth holds distances), or the frame's rgba
 * [P][4] with depth as svr_render_fwd writes it (the composited sum): then
 * D = depth / A where A >= min_alpha and A > 0, else no depth.
 * tsdf, weight: device float [n_grid], overwritten.  Points
 * and depths are read in fp32, projections and distances computed in fp64.
 * Errors: SVR_E_INVALID (n_grid outside [0, 2^31), trunc not finite > 0,
 * min_alpha not finite,
 * camera checks as for svr_preprocess, null arrays), SVR_E_HIP.
 *
 * svr_marching_cubes: triangles of the iso-surface field = iso over the
 * scene's voxels, each voxel one cell whose corner values are the field at
 * its 8 grid points (vox_grid).  A corner is above when field > iso; every
 * cell edge between an above and a below corner carries a vertex, keyed by
 * its two grid points (smaller index first) so that neighbouring cells share
 * it, at the linear interpolation of the corner positions (centre +- size/2)
 * at iso.  In each cell the crossings on every face are joined in pairs (four
 * crossings: two segments, each cutting off one above corner), oriented so
 * that the polygons' right-hand normals point to increasing field; each
 * polygon is a fan from its vertex with the smallest corner pair.  Cells with
 * a grid point of weight 0 (weight device float [n_grid], NULL: none) give no
 * triangles.  Uses scene->center, size, vox_grid, n_voxels, n_grid only.
 * field: device float [n_grid]; tri_keys: device int32 [max_triangles][3][2]
 * grid point pairs; tri_pos: device float [max_triangles][3][3];
 * n_triangles: device, receives the total count (which may exceed
 * max_triangles: then a cell whose triangles do not all fit writes none and
 * the caller retries with room for the count).  Triangle order varies from
 * call to call; each cell's triangles are consecutive and in table order.
 * Grid indices must lie in [0, n_grid) (not checked).
 * Errors: SVR_E_INVALID (sizes, non-finite iso, null arrays), SVR_E_HIP.   */
int svr_tsdf_fuse(const float* grid_pos, int64_t n_grid, const svr_camera* cams, int n_cams,
                  const float* depth, const float* rgba, float min_alpha, float trunc, float* tsdf,
                  float* weight, const uint32_t* order, void* stream);
int svr_marching_cubes(const svr_scene* scene, const float* field, const float* weight, float iso,
                       int64_t max_triangles, int32_t* tri_keys, float* tri_pos,
                       unsigned long long* n_triangles, const uint32_t* order, void* stream);
/* Visit order of the two calls above (`order`: NULL, or a device uint32
 * permutation of the grid points, resp. of the voxels, that the threads visit
 * in that order; results do not depend on it, speed does: points in
 * arbitrary order scatter the pixel and corner gathers).  svr_morton_keys
 * writes the Z-curve key of every point of pos (device float [3][n], x, y, z
 * rows) quantised to 1024 cells per axis of the cube [lo, lo + extent)
 * (lo: host float[3]; coordinates outside clamp to the border cells) into
 * keys (device uint64 [n], 30 bits) and 0..n-1 into values (device uint32
 * [n]); svr_radix_sort_pairs(keys, values, ..., bits = 30) then leaves the
 * order in values.  Entries of `order` outside [0, n) are skipped; a
 * permutation is not checked.  Errors: SVR_E_INVALID (n outside
 * [0, 2^32), non-finite lo, extent not finite > 0, null arrays), SVR_E_HIP. */
int svr_morton_keys(const float* pos, int64_t n, const float* lo, float extent, uint64_t* keys,
                    uint32_t* values, void* stream);
/* The cell table svr_marching_cubes uses (host memory, no GPU needed):
 * counts[case] triangles for case = sum over above corners c of 2^c;
 * verts[case][3 t + j] vertex j of triangle t as its corner pair a << 3 | b
 * (a < b).  counts: uint8 [256]; verts: uint8 [256][36].
 * Errors: SVR_E_INVALID (null arrays).                                     */
int svr_mesh_case_table(uint8_t* counts, uint8_t* verts);

/* Order ranks of the scene (build once per octpath set; Supp. B.1, B.2): the
 * sort key orders a tile's entries by (top 3L path bits XOR s * 0b001..001,
 * s).  rank[v*8 + s] is the position of pair (v, s) in that order over all 8N
 * pairs.  With it in svr_scene the per-frame key is tile << ceil(log2(8N)) |
 * rank: the same order (unique pair keys for max_level <= 15) in fewer radix
 * passes; svr_copy_sorted then returns keys of that form.
 * rank: device uint32 [8N].  scratch: device, 256-byte aligned,
 * >= svr_order_rank_scratch_bytes(n_voxels, max_level) (0 on invalid sizes).
 * Errors: SVR_E_INVALID, SVR_E_WORKSPACE, SVR_E_HIP.                         */
size_t svr_order_rank_scratch_bytes(int64_t n_voxels, int max_level);
int svr_build_order_ranks(const uint64_t* octpath, int64_t n_voxels, int max_level,
                          uint32_t* rank, void* scratch, size_t scratch_bytes, void* stream);

/* Corner adjacency of the grid points, a property of the scene topology
 * (build once per vox_grid): for grid point m, adj[adj_off[m] .. adj_off[m+1])
 * lists, in increasing order, the corner slots 8 v + c whose vox_grid entry is
 * m.  With it in svr_scene, svr_render_bwd forms grad_grid by a gather in a
 * fixed order (deterministic, no atomics) instead of scattering with atomics.
 *   vox_grid  device [N][8] (as in svr_scene); adj_off device [M+1]; adj device
 *   [8N]; scratch device >= svr_grid_adjacency_scratch_bytes(N, M).
 * Errors: SVR_E_INVALID, SVR_E_WORKSPACE, SVR_E_HIP.                         */
size_t svr_grid_adjacency_scratch_bytes(int64_t n_voxels, int64_t n_grid);
int svr_build_grid_adjacency(const int32_t* vox_grid, int64_t n_voxels, int64_t n_grid,
                             int32_t* adj_off, int32_t* adj, void* scratch, size_t scratch_bytes,
                             void* stream);

/* Static text of a status code; detail of the calling thread's last error. */
const char* svr_status_string(int status);
const char* svr_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SVRASTER_H */

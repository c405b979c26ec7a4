/*
 * fic.h -- fractal image encoding on AMD Instinct MI355X (gfx950).
 *
 * C ABI of libfic.so. It implements the encoder of Miar Naimi & Salarian,
 * "A Fast Fractal Image Compression Algorithm Using Predefined Values for
 * Contrast Scaling".
 *
 * Terms (Section 2 of the paper):
 *   range   a B x B block of the image; ranges tile the image.
 *   domain  a 2B x 2B block whose top-left corner lies on a grid of step L;
 *           it is decimated to B x B by taking 2x2 means.
 *   iso     one of 8 isometries applied to the decimated domain:
 *             t=0 identity            t=1 rotate 90 degrees clockwise
 *             t=2 rotate 180 degrees  t=3 rotate 270 degrees clockwise
 *             t=4..7 the left-right mirror of t=0..3.
 *           On a B x B block with row i and column c, t=1 places in[B-1-c][i]
 *           at (i, c), t=2 places in[B-1-i][B-1-c], and t=3 places
 *           in[c][B-1-i]. Mirrored forms read column B-1-c of the rotation.
 *   s, o    the contrast and offset of the affine map. s = k/10 with integer
 *           k in 0..10. The offset is that of eq. (3), o = mean(R) - s*mean(D).
 *   E       the distance of eq. (1), E = sum_i (s*d_i + o - r_i)^2.
 *
 * The search is exhaustive and exact. For every range the library returns
 * the candidate (domain, iso, contrast) with the smallest E. Exact integers
 * decide it, and ties go to the smallest (E, domain, iso, contrast index).
 * e_num = 1600 * n * E is an integer (n = B*B) and is reported exactly.
 *
 * Conventions for every entry point:
 *   - Pointers are DEVICE pointers unless marked [host].
 *   - The caller owns every buffer. The library never frees, keeps or
 *     aliases caller memory after a call returns.
 *   - Work is enqueued on `stream` (a hipStream_t, NULL = default stream).
 *     Outputs are valid once that stream has synchronised, unless the entry
 *     point says it synchronises itself.
 *   - Each call returns FIC_OK (0) or a negative fic_status. Arguments are
 *     validated on the host before any device work is queued; on an error
 *     nothing is queued. fic_last_error() then gives a message.
 *   - The library keeps internal device workspace per (device, stream). Calls
 *     on different streams may run concurrently; calls sharing one stream are
 *     ordered by it.
 */
#ifndef FIC_H
#define FIC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum fic_status {
    FIC_OK = 0,
    FIC_EINVAL = -1,    /* bad argument (shape, range, null pointer, ...) */
    FIC_ECAPACITY = -2, /* an output buffer is too small (see fic_encode_image) */
    FIC_EDEVICE = -3,   /* a HIP runtime error; the message carries its text */
    FIC_ENOMEM = -4     /* device workspace could not be allocated */
};

/* Largest image side the library accepts. */
#define FIC_MAX_SIDE 16384
/* Largest number of contrast values in one set. */
#define FIC_MAX_S 11

/* Best transform of one range block (24 bytes). */
typedef struct {
    int64_t e_num;  /* exact 1600 * n * E, E being eq. (1) at the optimum          */
    int32_t dom;    /* domain index on the level's unfiltered grid:                 */
                    /*   dom = (y / L) * gx + x / L, gx = (W - 2B) / L + 1          */
    uint8_t iso;    /* isometry t, 0..7                                             */
    uint8_t s_idx;  /* position of the chosen k in the contrast set                 */
    uint8_t k;      /* contrast numerator: s = k / 10                               */
    uint8_t flags;  /* FIC_FLAG_FALLBACK (learned encoder only), else 0             */
    int16_t q_o;    /* offset of eq. (3) rounded half up to an integer              */
    int16_t pad_;
    float E;        /* e_num / (1600 n) in FP32 (for reporting; e_num is exact)     */
} fic_match;

/* One leaf of the quadtree (32 bytes). */
typedef struct {
    int64_t e_num;  /* exact 1600 * n * E                                           */
    int32_t dom;    /* domain index on the level's unfiltered grid                  */
    int16_t y, x;   /* range top-left corner (pixels)                               */
    int16_t dy, dx; /* domain top-left corner (pixels)                              */
    int16_t q_o;    /* quantised offset                                             */
    uint8_t log2B;  /* range side B = 1 << log2B                                    */
    uint8_t iso;    /* isometry 0..7                                                */
    uint8_t k;      /* s = k / 10                                                   */
    uint8_t s_idx;  /* position of k in the level's contrast set                    */
    uint8_t level;  /* 0-based quadtree level                                       */
    uint8_t pad_[5];
} fic_code;

/* Per-level counters written by fic_encode_image (24 bytes). */
typedef struct {
    int64_t matches;  /* active ranges * pool domains * 8 isometries                */
    int32_t pool;     /* domains searched at this level                             */
    int32_t passed;   /* domains above the entropy threshold (= grid size if off)   */
    int32_t active;   /* ranges matched at this level                               */
    int32_t accepted; /* ranges whose transform was kept at this level              */
} fic_level_stats;

/* Encoder parameters (Sections 2 and 3). */
typedef struct {
    int32_t n_levels;       /* 1..4; level l has range side B0 >> l (>= 2)                */
    int32_t B0;             /* first-level range side, in {2, 4, 8, 16}                   */
    int32_t L[4];           /* domain step per level, >= 1                                */
    int32_t n_s[4];         /* contrast values per level, 1..FIC_MAX_S                    */
    int8_t s_k[4][12];      /* strictly increasing k in 0..10 per level (s = k/10)        */
    float rms_thresh;       /* keep a transform iff sqrt(E / n) <= rms_thresh;            */
                            /* the last level always keeps it                             */
    int32_t entropy_mode;   /* pool filter. 0: none. 1: keep domains whose 8-bin (p >> 5)  */
                            /* histogram entropy in bits exceeds entropy_bits (Section 3).*/
                            /* 2: keep domains whose pixel variance exceeds entropy_bits  */
                            /* (a variance filter, as a comparator)                       */
    float entropy_bits;     /* threshold of the filter (strict >): bits, or grey levels^2 */
    int32_t min_pool;       /* if fewer domains pass, use the min_pool domains of highest */
                            /* entropy (or variance) instead, ties to the lower index; >=1*/
} fic_params;

/*
 * Exhaustive matching at one level (Section 2; entropy filter of Section 3).
 *
 * img        uint8 image, H rows of W pixels, row stride `pitch` bytes.
 * B, L       range side (2, 4, 8 or 16) and domain step (>= 1). H and W must
 *            be multiples of B and at least 2B.
 * s_k, n_s   [host] 1..FIC_MAX_S strictly increasing contrast numerators k,
 *            each in 0..10 (s = k/10). The paper searches a sampled [0, 1]
 *            (Section 2) or a predefined per-step set (Section 3.1).
 * entropy_mode, entropy_bits, min_pool
 *            the domain-pool filter, as in fic_params. With entropy_mode = 0
 *            the pool is the whole grid.
 * range_yx   n_ranges pairs (y, x) of range top-left corners (multiples of B,
 *            inside the image), or NULL for the whole range grid in raster
 *            order (then n_ranges must equal (H/B)*(W/B)).
 * out        n_ranges fic_match records, in the order of range_yx.
 * pool_out   optional (may be NULL): receives the ascending domain indices
 *            searched; it must hold one int32 per grid domain.
 * pool_count optional (may be NULL): one device int32 receiving the pool size.
 *
 * Errors: FIC_EINVAL for bad shapes or arguments (range corners are checked
 * on the device; an out-of-image corner yields dom = -1 in its record).
 */
int fic_encode_level(const uint8_t* img, int32_t H, int32_t W, int32_t pitch, int32_t B,
                     int32_t L, const int8_t* s_k, int32_t n_s, int32_t entropy_mode,
                     float entropy_bits, int32_t min_pool, const int32_t* range_yx,
                     int32_t n_ranges, fic_match* out, int32_t* pool_out, int32_t* pool_count,
                     void* stream);

/* Matcher implementations for fic_encode_level_ex. */
enum fic_match_variant {
    FIC_MATCH_AUTO = 0,     /* the library's choice (what fic_encode_level uses)          */
    FIC_MATCH_VALU = 1,     /* dot4 correlation, exact 32/64-bit integer epilogue        */
    FIC_MATCH_MFMA_I8 = 2,  /* int8 MFMA screen of normalized domains (15-bit, two     */
                            /* bytes; the high byte first) against a bound of the range */
                            /* alone, candidates decided exactly from the integer data. */
                            /* AUTO takes it for the B = 8 contrast grid                */
    FIC_MATCH_FP32 = 3,     /* FP32 FMA correlation and FP32 E, no exact rescoring: a    */
                            /* comparator whose result may differ from the exact search  */
    FIC_MATCH_MFMA_F16 = 4  /* FP16 MFMA. Contrast grid at B = 8: the same screen with   */
                            /* FP16 normalized domains (one pass), exact decisions. One  */
                            /* or two values at B = 4, 8 or 16 (centred operands, FP32   */
                            /* accumulation exact: partial sums are integers below      */
                            /* 2^24): F exact in 32/64-bit integers; AUTO takes it there */
};

/*
 * fic_encode_level with an explicit matcher. FIC_MATCH_MFMA_I8, MFMA_F16 and
 * FIC_MATCH_FP32 need B = 8 and a contrast set 0, 1, ..., k1 with k1 >= 2;
 * the MFMA matchers also need a domain grid of fewer than 2^22 domains.
 * FIC_MATCH_MFMA_F16 also takes B = 4, 8 or 16 with one or two contrast values,
 * at least one nonzero, on a domain grid of fewer than 2^21 domains
 * (FIC_EINVAL otherwise; AUTO then takes the VALU matcher). VALU, MFMA_I8,
 * MFMA_F16 and AUTO return the exact result.
 * FP32 returns its own FP32 argmin with its FP32 E in `E` and, in e_num, the
 * exact 1600 n E of the candidate it chose.
 */
int fic_encode_level_ex(const uint8_t* img, int32_t H, int32_t W, int32_t pitch, int32_t B,
                        int32_t L, const int8_t* s_k, int32_t n_s, int32_t entropy_mode,
                        float entropy_bits, int32_t min_pool, const int32_t* range_yx,
                        int32_t n_ranges, fic_match* out, int32_t* pool_out, int32_t* pool_count,
                        int32_t variant, void* stream);

/*
 * Measured peak rates of this device, the denominators of roofline
 * fractions (not part of the paper's method). Each probe keeps one unit busy
 * with independent chains over the whole chip, times 5 launches after 2
 * warm-ups with HIP events on `stream`, and synchronises. *rate receives:
 *   FIC_PEAK_VALU_FMA  32-bit multiply-add rate (fp32 FMA, unpacked), ops/s
 *                      (2 per lane per instruction)
 *   FIC_PEAK_DOT2      v_dot2_i32_i16 rate, ops/s (4 per lane per instruction)
 *   FIC_PEAK_MFMA_F16  v_mfma_f32_16x16x32_f16 rate, flop/s
 *   FIC_PEAK_MFMA_I8   v_mfma_i32_16x16x64_i8 rate, ops/s
 *   FIC_PEAK_HBM_COPY  device-to-device copy of 1 GiB, bytes read + written
 *                      per second (allocates and frees 2 GiB)
 */
enum fic_peak { FIC_PEAK_VALU_FMA = 0, FIC_PEAK_DOT2 = 1, FIC_PEAK_MFMA_F16 = 2, FIC_PEAK_MFMA_I8 = 3,
                FIC_PEAK_HBM_COPY = 4 };
int fic_peak_probe(int32_t what, void* stream, double* rate);

/* Device scratch of fic_encode_level_noalloc, per GPU (64 MiB). */
#define FIC_NOALLOC_SCRATCH_BYTES (64u << 20)

/*
 * fic_encode_level with no device allocation, for callers that cannot
 * allocate: code under hipGraph stream capture, serving loops that must not
 * call hipMalloc, harnesses that forbid it. Arguments, outputs and results
 * are those of fic_encode_level (FIC_MATCH_AUTO matcher): the same kernels
 * run, bit for bit the same records.
 *
 * Every buffer the search needs beyond the caller's inputs and outputs
 * (control blocks, entropy table, pool keys and lists, domain moments,
 * per-chunk partial results, active lists) lives in one array of
 * FIC_NOALLOC_SCRATCH_BYTES bytes in each GPU's memory, held until the
 * process ends. The call allocates nothing: no hipMalloc, hipFree or event
 * creation; it queues kernels and device-to-device copies on `stream`.
 *
 * Limit: a level whose buffers exceed the array is rejected with FIC_EINVAL
 * before anything is queued; the message gives the bytes it would need. The
 * needs grow with the domain grid (28 + 2n bytes per grid domain, n = B*B;
 * 28 + 4n where the FP16 small-set matcher runs; about 360 at B = 8 with a
 * contrast grid 0..k1) and with n_ranges (about 85 bytes each for large
 * range lists). For example 512x512 at B = 2, L = 1 (259081 domains, 65536
 * ranges) takes about 15 MiB and 1024x1024 at B = 2, L = 1 about 60 MiB;
 * 1024x1024 at B = 8, L = 2 with the 11-value grid does not fit.
 *
 * Sharing: all calls on one GPU use that GPU's one array, which keeps the
 * last call's contents (each call first resets the parts that must start
 * at zero). Calls that overlap in time on one GPU, on any streams, race and
 * give undefined results: order them (one stream, or events). The first call
 * on each GPU resolves the array's address and uploads the entropy table
 * with a synchronous copy, so make it outside stream capture.
 */
int fic_encode_level_noalloc(const uint8_t* img, int32_t H, int32_t W, int32_t pitch, int32_t B,
                             int32_t L, const int8_t* s_k, int32_t n_s, int32_t entropy_mode,
                             float entropy_bits, int32_t min_pool, const int32_t* range_yx,
                             int32_t n_ranges, fic_match* out, int32_t* pool_out,
                             int32_t* pool_count, void* stream);

/*
 * Quadtree encoder (Section 2; the three cases at the end of Section 3.1).
 * Level 0 matches every B0 x B0 range. A range whose best transform has
 * RMS error above p->rms_thresh is split into its four quadrants (top-left,
 * top-right, bottom-left, bottom-right) for the next level. The last level
 * keeps everything.
 *
 * codes      capacity fic_code records. Codes are written level by level. Within a level
 *            they follow the active list: raster order at level 0, and below it
 *            the four children of each split range in the order of their parents.
 * n_codes    one device int32. It receives the number of codes the image
 *            needs, even when that exceeds `capacity`; records past capacity
 *            are dropped. After synchronising, n_codes > capacity means the
 *            buffer was too small.
 * stats      optional (may be NULL): p->n_levels fic_level_stats records.
 *
 * Errors: FIC_EINVAL (shapes, parameters); FIC_ECAPACITY when capacity is
 * below (H/B0)*(W/B0), the fewest codes any image needs.
 */
int fic_encode_image(const uint8_t* img, int32_t H, int32_t W, int32_t pitch,
                     const fic_params* p, fic_code* codes, int32_t capacity, int32_t* n_codes,
                     fic_level_stats* stats, void* stream);

/*
 * Decoder for the reconstructions of Section 4 (the paper does not describe
 * one). Starts from a uniform grey 128 image and applies the code's map
 * `iters` times. Each iteration rebuilds every leaf from the previous image:
 * value = (k/10) * T_iso(2x2 mean of the domain) + q_o, rounded half up and
 * clamped to 0..255, in exact integer arithmetic.
 *
 * codes, n_codes  leaves that tile the H x W image exactly.
 * out             uint8 image, row stride out_pitch (>= W).
 * Synchronises `stream` before returning. Codes that do not tile the image,
 * or that point outside it, give FIC_EINVAL.
 */
int fic_decode(const fic_code* codes, int32_t n_codes, int32_t H, int32_t W, int32_t iters,
               uint8_t* out, int32_t out_pitch, void* stream);

/*
 * Sum of squared differences between two uint8 images (for PSNR).
 * sse: one device uint64.
 */
int fic_sse(const uint8_t* a, int32_t pitch_a, const uint8_t* b, int32_t pitch_b, int32_t H,
            int32_t W, uint64_t* sse, void* stream);

/*
 * Predefined contrast values estimated from low-entropy ranges (abstract;
 * Section 3.1). Runs the plain method (k = 0..10, no domain filter) through
 * the quadtree of p (n_levels, B0, L, rms_thresh). At each level it takes the
 * kept ranges whose 8-bin entropy is <= p->entropy_bits, and returns the mean
 * of their best k rounded half up. A level without such a range gets -1.
 * k_out: [host] p->n_levels int8. Synchronises `stream`.
 */
int fic_calibrate_s(const uint8_t* img, int32_t H, int32_t W, int32_t pitch,
                    const fic_params* p, int8_t* k_out, void* stream);

/* Device time of one kernel label, from HIP events (40 bytes). */
typedef struct {
    char name[24];     /* kernel label, e.g. "match_b2" or "pool_score"             */
    int32_t launches;  /* launches recorded                                          */
    int32_t pad_;
    double total_ms;   /* summed time between the events around each launch          */
} fic_kernel_time;

/*
 * Profiling hooks (measurement only; the encoder never needs them).
 * fic_profile_begin clears earlier records and starts recording. Every later
 * launch of a library kernel, on any stream, is then bracketed by two HIP
 * events on its stream.
 * fic_profile_end stops recording and waits for the recorded events. It sums
 * the intervals per kernel label into out[0 .. max-1], longest total first,
 * and writes the number of labels to *n_out (out and n_out may be NULL).
 * Process-wide; not meant to run while another thread encodes.
 */
int fic_profile_begin(void);
int fic_profile_end(fic_kernel_time* out, int32_t max, int32_t* n_out);

/*
 * fic_encode_image with two optional outputs for the bitstream:
 * flags  device uint32 bitmap (may be NULL): bit sum_{l'<l} active_l' + q is
 *        set iff active range q of level l was split (levels but the last).
 *        Size: one bit per possible range of every level but the last, i.e.
 *        ceil(sum_l<n_levels-1 (H/B_l)(W/B_l) / 32) words; cleared here.
 * pools  device int32 (may be NULL; used only with a pool filter): level l's
 *        ascending pool list at offset sum_{l'<l} grid_l' (grid_l = domains
 *        of level l's unfiltered grid), stats[l].pool entries long.
 */
int fic_encode_image_ex(const uint8_t* img, int32_t H, int32_t W, int32_t pitch, const fic_params* p,
                        fic_code* codes, int32_t capacity, int32_t* n_codes, fic_level_stats* stats,
                        uint32_t* flags, int32_t* pools, void* stream);

/*
 * Bitstream of a quadtree encode (the paper reports compression ratios in
 * Section 4 without a bit allocation; this fixed-length layout is the reading
 * used here). Bit b is bit (b mod 8) of byte b / 8.
 *   header  magic 0xF1C5 (16), version 1 (8), H (16), W (16), B0 (5),
 *           n_levels (3); per level: L (16), n_s (4), the k values (4 each),
 *           listed (1); if listed (a pool filter is on, the level has leaves
 *           and 24 + P bits(grid) + leaves bits(P) < leaves bits(grid)): pool
 *           size P (24), then the P ascending grid indices (bits(grid) each).
 *   flags   every level but the last: one bit per active range, active-list
 *           order, 1 = split into TL, TR, BL, BR.
 *   leaves  code order: domain (position in the level's pool, bits(P); the
 *           grid index when not listed), isometry (3), contrast index
 *           (bits(n_s)), offset q_o (9, two's complement).
 * bits(x) = ceil(log2 x) for x >= 2, else 0.
 *
 * fic_stream_bound: bytes that always suffice (a multiple of 4), or -1.
 * fic_pack_stream: codes, stats, flags and pools of one fic_encode_image_ex
 *   call (device); out is device memory, 4-byte aligned, capacity a multiple
 *   of 4 bytes. *n_bytes (device int64) receives the stream length; bytes
 *   beyond capacity are not written.
 * fic_unpack_stream: [host] reader. Fills up to capacity [host] codes (e_num
 *   = -1: not stored), sets *n_codes to the number in the stream, and *H, *W.
 *   FIC_EINVAL on a malformed stream, FIC_ECAPACITY if capacity is too small.
 */
int64_t fic_stream_bound(int32_t H, int32_t W, const fic_params* p);
int fic_pack_stream(const fic_code* codes, int32_t n_codes, int32_t H, int32_t W, const fic_params* p,
                    const fic_level_stats* stats, const uint32_t* flags, const int32_t* pools,
                    uint8_t* out, int64_t capacity, int64_t* n_bytes, void* stream);
int fic_unpack_stream(const uint8_t* data, int64_t n_bytes, fic_code* codes, int32_t capacity,
                      int32_t* n_codes, int32_t* H, int32_t* W);

/*
 * Batched quadtree encoder. It encodes n images of possibly different sizes
 * with the same parameters. Every level of every image runs in shared kernel
 * launches, which are captured once into a hipGraph; fic_batch_run replays
 * that graph.
 *
 * imgs, H, W, pitch  [host] arrays of n: device image pointers and their
 *                    shapes, as in fic_encode_image. The images must stay
 *                    valid and at the same addresses while the batch exists.
 * codes, code_offset codes is a device buffer. code_offset is a [host] array
 *                    of n+1 entries: image i writes its codes to
 *                    codes[code_offset[i] .. code_offset[i+1]). Each range
 *                    must hold at least (H/B0)*(W/B0) codes (FIC_ECAPACITY).
 * n_codes            device int32[n]: codes needed per image, as in
 *                    fic_encode_image.
 * stats              optional device fic_level_stats[n * p->n_levels].
 * The batch owns one workspace per image and a private stream for capture.
 * Replays on one batch must not overlap. Only the device memory is per call.
 * A new batch runs in the level form (FIC_BATCH_LEVELS); fic_batch_set_form
 * selects the persistent form.
 */
typedef struct fic_batch fic_batch;
int fic_batch_create(int32_t n, const uint8_t* const* imgs, const int32_t* H, const int32_t* W,
                     const int32_t* pitch, const fic_params* p, fic_code* codes,
                     const int64_t* code_offset, int32_t* n_codes, fic_level_stats* stats,
                     fic_batch** out);
/* Replay the captured encode on `stream` (asynchronous). */
int fic_batch_run(fic_batch* b, void* stream);
/*
 * The same kernels with the same launch shapes, queued one by one on
 * `stream` instead of through the graph (asynchronous). Used to time each
 * kernel between fic_profile_begin and fic_profile_end.
 */
int fic_batch_run_eager(fic_batch* b, void* stream);
/*
 * Tile shape of the batch: pool domains per matcher chunk for each level
 * ([host] p->n_levels values, 0 = the library default). Set it directly, or
 * let fic_batch_autotune choose it.
 */
int fic_batch_set_chunks(fic_batch* b, const int32_t* chunks);
int fic_batch_get_chunks(const fic_batch* b, int32_t* chunks);

/* How a batch's encode runs (the quadtree of Section 2 either way; the
   codes, counts and statistics are identical). */
enum fic_batch_form {
    /* per level, shared launches over all images: pools, matcher, keep/split
       decisions, compaction of the next level's active list */
    FIC_BATCH_LEVELS = 0,
    /* the pools of every level, then ONE persistent kernel: resident
       workgroups drain a device queue of (image, level, range tile) tasks,
       matching each tile over its level's pool, deciding keep/split, and
       queueing the four children of every split range on the device (a tile
       of the next level is queued as soon as it fills); then an ordered
       compaction of the results into codes */
    FIC_BATCH_PERSISTENT = 1
};
/*
 * Select the form and, for the persistent form, its tile shape: tiles[l]
 * ranges per tile at level l ([host] p->n_levels values or NULL; 0 = the
 * library default; a multiple of the level matcher's range block, at most
 * 256) and the number of resident workgroups (0 = every one that fits on
 * the device; larger values are clamped to that). Rebuilds the graph; on an
 * error the previous form is kept. Levels whose automatic matcher is an
 * MFMA grid form (B = 8 with a contrast grid) run the VALU matcher in the
 * persistent form; results are the same (both exact).
 */
int fic_batch_set_form(fic_batch* b, int32_t form, const int32_t* tiles, int32_t workgroups);
/* The current form, tile shape (ranges per tile per level, 0 for the level
   form) and workgroup count (0 for the level form); pointers may be NULL. */
int fic_batch_get_form(const fic_batch* b, int32_t* form, int32_t* tiles, int32_t* workgroups);
/*
 * Autotuner of the current form, timing `reps` graph replays on `stream` per
 * candidate and keeping the fastest. Level form: coordinate descent over each
 * level's chunk size. Persistent form: coordinate descent over each level's
 * ranges per tile (1, 2, 4 or 8 matcher blocks), then over the resident
 * workgroups per compute unit. The choice is cached in cache_path (JSON
 * lines; may be NULL), keyed by GPU architecture, HIP runtime version, image
 * sizes, parameters and form. A cached entry is applied without tuning.
 * *best_ms (may be NULL) receives the mean replay time. Synchronises `stream`.
 */
int fic_batch_autotune(fic_batch* b, void* stream, int32_t reps, const char* cache_path,
                       float* best_ms);
int fic_batch_destroy(fic_batch* b);

/*
 * Learned domain proposal: an extension of the exhaustive search of Section 2
 * for 8 x 8 ranges. A network f (64 -> 256 -> 256 -> 64, ReLU after the first
 * two layers, fp16 weights, fp32 accumulation) embeds a block vector x (the
 * block's 64 values -- range pixels, or a domain's 2x2 sums -- mean removed
 * and scaled to unit norm, zero for a constant block) as
 *     g(x) = S / |S|,  S = sum over the 8 isometries T_t of f(T_t x),
 * which is invariant under the isometries. The k domains whose embeddings
 * are most similar to a range's (the integer dot product of their int8 codes,
 * as fic_topk_similar defines it) are its proposals. They are
 * matched exactly (eq. (1) with the offset of eq. (3), all isometries and
 * contrast values, ties as in the exhaustive matcher). A range whose best
 * proposal fails the RMS test of Section 2 (E > rms^2 n) is matched against
 * every domain instead.
 *
 * Parameters, flat fp32, FIC_MLP_PARAMS values: W1 [256][64], b1 [256],
 * W2 [256][256], b2 [256], W3 [64][256], b3 [64], each W stored (out, in).
 * A fic_mlp owns device copies of them, the Adam moments and scratch space.
 * Calls on one fic_mlp must not overlap. Its entry points run on the device
 * that was current at fic_mlp_create.
 */
#define FIC_MLP_PARAMS 98880
#define FIC_FLAG_FALLBACK 1 /* fic_match.flags: the exhaustive search decided */
typedef struct fic_mlp fic_mlp;
/* init: [host] FIC_MLP_PARAMS finite values. tau > 0: similarity scale of the
 * training loss. Synchronous. */
int fic_mlp_create(const float* init, float tau, fic_mlp** out);
int fic_mlp_destroy(fic_mlp* m);
/* Current parameters into [host] out (FIC_MLP_PARAMS floats). Synchronises the device. */
int fic_mlp_get_params(const fic_mlp* m, float* out);
/*
 * Embeddings of n blocks into out (device, fp16 bit patterns, [n][64]).
 * kind 0: 8 x 8 ranges; list = device int32 [n][2] corners (y, x), or NULL
 *         for the whole range grid in raster order (n = (H/8)(W/8)).
 * kind 1: 16 x 16 domains on the step-L grid; list = device int32 [n] domain
 *         indices, or NULL for every domain (n = grid size).
 * H, W multiples of 8 and >= 16. A corner or index outside the image gives
 * the embedding of a constant block.
 */
int fic_mlp_embed(fic_mlp* m, const uint8_t* img, int32_t H, int32_t W, int32_t pitch, int32_t kind,
                  int32_t L, const int32_t* list, int32_t n, uint16_t* out, void* stream);
/*
 * Training loss and gradient. For the n_ranges ranges at range_yx (device
 * int32 [n][2], or NULL for the whole grid) and every domain of the step-L
 * grid: the mean over ranges of the softmax cross-entropy of the similarities
 * g(r) . g(d_j) / tau against labels (device int32 [n], a domain index;
 * a label outside the grid contributes nothing). loss_out: device float
 * (may be NULL). grad_out: device float [FIC_MLP_PARAMS] (may be NULL; the
 * gradient is also kept for fic_mlp_adam).
 */
int fic_mlp_loss_grad(fic_mlp* m, const uint8_t* img, int32_t H, int32_t W, int32_t pitch,
                      int32_t L, const int32_t* range_yx, const int32_t* labels, int32_t n_ranges,
                      float* loss_out, float* grad_out, void* stream);
/* One Adam step (bias-corrected) with grad (device float [FIC_MLP_PARAMS]) or,
 * when grad is NULL, the last gradient fic_mlp_loss_grad computed. */
int fic_mlp_adam(fic_mlp* m, const float* grad, float lr, float beta1, float beta2, float eps,
                 void* stream);
/* fic_mlp_loss_grad then fic_mlp_adam(lr, 0.9, 0.999, 1e-8). */
int fic_mlp_train_step(fic_mlp* m, const uint8_t* img, int32_t H, int32_t W, int32_t pitch,
                       int32_t L, const int32_t* range_yx, const int32_t* labels,
                       int32_t n_ranges, float lr, float* loss_out, void* stream);
/*
 * For each of nq query rows (device fp16 [nq][64], 16-byte aligned), the k
 * (1..32) key rows (device fp16 [nk][64], 16-byte aligned) with the largest
 * similarity, best first, ties to the lower key index: idx device int32
 * [nq][k] (-1 past nk), score device float [nq][k] (may be NULL; -inf past
 * nk). The similarity is the dot product of int8 codes q = rint(x s), with
 * one scale s = 127 / max |x| over the queries and the keys together (fp32
 * arithmetic; s = 0 when every value is 0): an integer, returned exactly as a
 * float. This is the proposal step of the learned form (an extension of the
 * exhaustive search of Section 2). m provides scratch space only.
 */
int fic_topk_similar(const uint16_t* q, int32_t nq, const uint16_t* keys, int32_t nk, int32_t k,
                     int32_t* idx, float* score, fic_mlp* m, void* stream);
/*
 * Learned-proposal encode of the full 8 x 8 range grid (raster order) with
 * domains on the step-L grid, contrast values s_k / 10 ([host] n_s values)
 * and topk proposals (1..32) per range. out: device fic_match [(H/8)(W/8)];
 * ranges decided by the exhaustive fallback carry FIC_FLAG_FALLBACK.
 * proposals_out: device int32 [(H/8)(W/8)][topk] or NULL; n_fallback: device
 * int32 or NULL.
 */
int fic_encode_level_learned(fic_mlp* m, const uint8_t* img, int32_t H, int32_t W, int32_t pitch,
                             int32_t L, const int8_t* s_k, int32_t n_s, int32_t topk,
                             float rms_thresh, fic_match* out, int32_t* proposals_out,
                             int32_t* n_fallback, void* stream);
/* Codes (level 0) of a full range grid's matches, for fic_decode. */
int fic_level_codes(const fic_match* m, int32_t H, int32_t W, int32_t B, int32_t L, fic_code* codes,
                    void* stream);

/*
 * Distribution of the optimal contrast, for choosing predefined values per
 * quadtree step (Section 3.1, Fig. 3). Encodes the image with the plain
 * method (11 values, no pool filter, p's levels, steps and RMS threshold) and
 * adds 1 to hist[l][k] (device uint64 [4][11], not cleared: calls accumulate
 * over an image set) for every kept leaf of level l with contrast k/10 -- all
 * of them, or with low_entropy_only only those whose range has 8-bin entropy
 * <= p->entropy_bits. Synchronises `stream`.
 */
int fic_s_histogram(const uint8_t* img, int32_t H, int32_t W, int32_t pitch, const fic_params* p,
                    int32_t low_entropy_only, uint64_t* hist, void* stream);
/*
 * [host] Predefined values from such histograms ([host] uint64 [n_levels][11]):
 * per level the most frequent k, plus the second most frequent when its count
 * is at least second_frac of the first (ties to the smaller k); s_k [4][2]
 * ascending, n_s[l] = 1 or 2, or 0 for an empty histogram.
 */
int fic_select_s(const uint64_t* hist, int32_t n_levels, float second_frac, int8_t* s_k, int32_t* n_s);

/* Message for the last non-zero return on this thread. */
const char* fic_last_error(void);

/* ABI version (major * 100 + minor). */
int fic_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FIC_H */

/*
 * fftb.h -- C ABI of the MI355X plane-wave sphere<->grid 3D FFT library.
 *
 * The library computes, for a batch of bands, the two transforms that move
 * plane-wave coefficients between a cutoff sphere and a dense cuboid grid:
 *
 *   sphere_to_grid (inverse):  psi_b(x,y,z) = sum_{g in sphere} c_b(g) *
 *        exp(+2*pi*i*(mx*x/nx + my*y/ny + mz*z/nz))            (unnormalised)
 *   grid_to_sphere (forward):  c_b(g) = (1/N) * sum_{x,y,z} psi_b(x,y,z) *
 *        exp(-2*pi*i*(mx*x/nx + my*y/ny + mz*z/nz)),  N = nx*ny*nz
 *
 * The plane-wave expansion and the inclusive energy cutoff that defines the
 * sphere are in Section 2.2 of the paper; the DFT matrix and its sign
 * (negative exponent = forward) in Section 2.1; the offset-array description of
 * a sphere projected on the xy-plane and the batch dimension placed first
 * (fastest in memory) in Section 3.3; the create / execute / clean-up object
 * model in Section 3.1. The padding is applied one axis at a time and fused
 * with the 1D transforms (Section 2.2): z-transforms run only on the occupied
 * (x,y) columns, y-transforms only on the occupied x-slab, x-transforms on the
 * full grid.
 *
 * Layouts (all complex values interleaved (re, im), double for FFTB_C128 and
 * float for FFTB_C64):
 *   sphere buffer: for each sphere s in order, S_s[g][b] -- coefficient g in
 *                  map order, band b fastest; Ns_s * nbands_s values.
 *   grid buffer:   for each sphere s in order, G_s[z][y][x][b] -- band
 *                  fastest, then x, then y, then z; N * nbands_s values.
 * A map entry is the wrapped linear grid index x + nx*(y + ny*z), where
 * x = mx mod nx, y = my mod ny, z = mz mod nz for the signed frequency
 * (mx, my, mz). Entries must be unique and in [0, N). Any order is accepted.
 *
 * Ownership: the caller owns all data buffers (device memory). The plan copies
 * the maps at create time and owns its device tables and scratch (allocated at
 * create, freed at destroy).
 *
 * Streams: execute calls enqueue work on the given HIP stream (hipStream_t,
 * NULL = default stream) and return without synchronising. Buffers must stay
 * valid until that work completes. A plan holds one scratch buffer, so calls
 * on one plan must not overlap in time (serialise them on one stream).
 *
 * Errors: every entry point returns an fftb_status. No C++ exception crosses
 * the ABI. fftb_last_error() gives a thread-local detail message for the last
 * failing call on the calling thread.
 *
 * Environment: FFTB_LOG (set, not "0") prints a plan summary on stderr at plan
 * creation; FFTB_MAX_DEVICE_BYTES bounds the device memory of one plan (a plan
 * that would exceed it fails with FFTB_ERR_NOMEM before any device call).
 */
#ifndef FFTB_H
#define FFTB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FFTB_OK = 0,
  FFTB_ERR_INVALID = -1,      /* bad argument: null pointer, bad size, duplicate or out-of-range index */
  FFTB_ERR_UNSUPPORTED = -2,  /* a pattern the library does not implement (prime factor > 5, ...) */
  FFTB_ERR_NOMEM = -3,        /* device allocation failed */
  FFTB_ERR_HIP = -4           /* a HIP runtime call or kernel launch failed */
} fftb_status;

typedef enum {
  FFTB_C128 = 0,  /* complex double */
  FFTB_C64 = 1    /* complex float: FP32 arithmetic, FP64-generated twiddles stored as hi+lo FP32 */
} fftb_dtype;

/* Plan flags (bitwise OR). */
enum {
  FFTB_PLAN_PLAIN = 0,       /* one launch per kernel per call, grid sized to the work */
  FFTB_PLAN_BATCHED = 1,     /* persistent kernels walking a device work list over all spheres */
  FFTB_PLAN_AUTOTUNE = 2,    /* time candidate tilings at create time and keep the fastest per
                                direction; results are cached in the file named by the
                                FFTB_TUNE_CACHE environment variable (default: none). The
                                trials share one scratch buffer, try at most
                                FFTB_TUNE_MAX_CANDIDATES tilings per direction (default 16),
                                stop after FFTB_TUNE_SECONDS (default 60) keeping the best so
                                far, and print one progress line per trial on stderr */
  FFTB_PLAN_GRAPH = 4,       /* replay each direction as a captured hipGraph */
  FFTB_PLAN_HOST_ONLY = 8,   /* build and validate the host tables only; no device work (testing) */
  FFTB_PLAN_MFMA = 16        /* FFTB_C64 only: radix-16 stages as FP32 MFMA dense products (the
                                inverse fold's length-16 transforms of band-inner plans with y
                                classes of 16, the in-lane DFT_16 of 128-point register lines);
                                UNSUPPORTED for a plan with neither */
};

typedef struct fftb_plan_s* fftb_plan; /* opaque */

/* One k-point's sphere (Section 2.2: the coefficients kept inside the cutoff;
 * Section 3.3: the offset array that locates them in the grid). */
typedef struct {
  int64_t n_coeffs;    /* Ns >= 1 */
  const int32_t* map;  /* host pointer, Ns wrapped linear indices (see above) */
  double kpt[3];       /* k-point in fractional grid units; metadata only -- it
                          enters the transform only through which G the map holds */
  int32_t nbands;      /* >= 1 bands sharing this map */
} fftb_sphere;

/* Tiling of one direction. A zero field means "library default". */
typedef struct {
  int32_t band_chunk;   /* bands per workgroup tile, power of two, 1..64; path 3 takes one
                           128-byte piece (16 complex64 / 8 complex128 bands), and for the
                           complex64 inverse also half of one (8: the plane kernel's x lines
                           over twice the positions, the column kernel on whole pieces) */
  int32_t y_classes;    /* n1: the plane kernel splits the y index into n1 residue classes; divides ny */
  int32_t x_rows;       /* rows per x-transform batch (LDS-stage path only) */
  int32_t col_tile;     /* columns per column-kernel task */
  int32_t threads;      /* plane-kernel workgroup size: 64, 128, 256 or 512 */
  int32_t path;         /* 0 = choose, 1 = LDS-stage kernels, 2 = register-line kernels
                           (bands across lanes, a line over 1..16 lanes), 3 = band-inner lines
                           (one 128-byte piece of bands per row of 16 lanes, a line over the
                           rows of a wavefront); UNSUPPORTED where no shape fits */
  int32_t acc;          /* forward: 0 = choose, 1 = column accumulators in LDS (the plane's
                           columns split over workgroups), 2 = accumulators in global memory,
                           3 = one task per y class writing class partials that a combine
                           kernel turns into columns (a length-n1 DFT over the classes;
                           one split). inverse, path 3: 0 = choose, 1 = one y class per plane
                           task, 2 = two classes r and r + n1/2 per task, folded from the same
                           reads of the plane's columns (even n1, classes of 16) */
  int32_t splits;       /* forward only: column splits per (plane, chunk), 1..8 */
  int32_t lanes;        /* register path: lanes per transform line (x lines of the plane
                           kernel, z lines of the column kernel): 0 = choose, or 1, 4, 8, 16
                           where a line shape of that many lanes is compiled */
} fftb_dir_tuning;

/* Tiling knobs of both directions (they are chosen and tuned independently). */
typedef struct {
  fftb_dir_tuning inv;  /* sphere_to_grid */
  fftb_dir_tuning fwd;  /* grid_to_sphere */
} fftb_tuning;

/* Summary of a plan. */
typedef struct {
  int32_t dims[3];
  int32_t nspheres;
  int32_t dtype;
  uint32_t flags;
  int64_t total_coeffs;        /* sum of Ns */
  int64_t sphere_elems;        /* sum of Ns * nbands: length of the sphere buffer in complex values */
  int64_t grid_elems;          /* sum of N * nbands: length of the grid buffer in complex values */
  int64_t total_columns;       /* sum over spheres of occupied (x,y) columns */
  int32_t max_columns;
  int32_t max_slab;            /* max over spheres of occupied x planes */
  int64_t workspace_bytes;     /* device scratch + tables held by the plan */
  int32_t radix_x[8], radix_y[8], radix_z[8]; /* per-axis radix plan, 0-terminated */
  fftb_tuning tuning;          /* the tiling in use */
  int32_t autotuned;           /* 1 if the tiling came from timed trials, 2 if from the tuning cache */
} fftb_plan_info;

/*
 * Create a plan for nspheres spheres on a grid dims = {nx, ny, nz}.
 *   out      -- receives the plan (set to NULL on failure)
 *   dims     -- host pointer, 3 values >= 1 whose prime factors are 2, 3, 5 only
 *               (else FFTB_ERR_UNSUPPORTED)
 *   spheres  -- host array of nspheres descriptors; maps are copied
 *   dtype    -- FFTB_C128 or FFTB_C64
 *   flags    -- FFTB_PLAN_* bits
 *   tuning   -- optional host pointer; NULL or zero fields = defaults (ignored
 *               for fields the autotuner chooses when FFTB_PLAN_AUTOTUNE is set)
 *   stream   -- hipStream_t used for table uploads and autotuning trials
 * Returns FFTB_ERR_INVALID for a null pointer, nspheres < 1, Ns < 1, nbands < 1,
 * a map index outside [0, N) or a duplicate index; FFTB_ERR_UNSUPPORTED for a
 * dimension with a prime factor above 5 or a tiling that does not fit; HIP or
 * allocation failures as FFTB_ERR_HIP / FFTB_ERR_NOMEM.
 */
fftb_status fftb_plan_create(fftb_plan* out, const int32_t dims[3],
                             const fftb_sphere* spheres, int32_t nspheres,
                             fftb_dtype dtype, uint32_t flags,
                             const fftb_tuning* tuning, void* stream);

/* The classic batched cuboid transform (the paper's first API example,
 * Section 3.2, a 3D FFT of a batch of cuboid grids): a plan whose single
 * "sphere" is every grid point in G[z][y][x] order, so that both buffers hold
 * N * nbands values in the grid layout. sphere_to_grid is then the
 * unnormalised inverse 3D DFT of the batch and grid_to_sphere the forward one
 * scaled by 1/N. Arguments and errors as for fftb_plan_create (nbands >= 1). */
fftb_status fftb_plan_create_cuboid(fftb_plan* out, const int32_t dims[3], int32_t nbands,
                                    fftb_dtype dtype, uint32_t flags,
                                    const fftb_tuning* tuning, void* stream);

/* Inverse transform (sphere -> grid) of every band of every sphere.
 * sphere_in: device pointer, info.sphere_elems complex values (read only).
 * grid_out:  device pointer, info.grid_elems complex values (fully written).
 * The two buffers must not overlap. */
fftb_status fftb_sphere_to_grid(fftb_plan plan, const void* sphere_in, void* grid_out,
                                void* stream);

/* Forward transform (grid -> sphere), scaled by 1/N.
 * grid_in:    device pointer, info.grid_elems complex values (not modified).
 * sphere_out: device pointer, info.sphere_elems complex values (fully written). */
fftb_status fftb_grid_to_sphere(fftb_plan plan, const void* grid_in, void* sphere_out,
                                void* stream);

/* Real-space step between the two transforms (Section 1 of the paper: the
 * Kohn-Sham wavefunctions, and operations that are cheaper in real space):
 * for every band, psi = sphere_to_grid(c); psi(x,y,z) *= V(x,y,z);
 * c' = grid_to_sphere(psi). The multiply is fused into the stores of the
 * inverse plane kernel, so the step moves the bytes of one round trip.
 * potential:  device pointer, N real values (double for FFTB_C128, float for
 *             FFTB_C64) in V[z][y][x] order, shared by all bands and spheres.
 * grid_work:  device pointer, info.grid_elems complex values; receives V*psi.
 * sphere_in / sphere_out: as for the two transforms (must not overlap grid_work). */
fftb_status fftb_apply_potential(fftb_plan plan, const void* sphere_in, const void* potential,
                                 void* grid_work, void* sphere_out, void* stream);

/* Bytes of the static device scratch that fftb_sphere_to_grid_static uses. */
#define FFTB_STATIC_SCRATCH_BYTES (64u << 20)

/* For callers that cannot allocate device memory when they transform (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): fftb_sphere_to_grid with the plan's column scratch replaced by
 * a static device array of FFTB_STATIC_SCRATCH_BYTES (64 MiB) that the library
 * holds on every GPU it runs on until the process ends. The call allocates
 * nothing (no hipMalloc, no events, no graph instantiation, even for plans
 * created with FFTB_PLAN_GRAPH: it enqueues the kernels directly). Arguments,
 * layouts and results as for fftb_sphere_to_grid. Returns FFTB_ERR_UNSUPPORTED,
 * without enqueuing anything, when the plan's inverse column scratch (its
 * column slots x nz x band stride x value size) exceeds the static array.
 * Every call on one GPU shares that GPU's array: the call clears the part it
 * needs zero before its kernels run, and calls that overlap in time on one GPU
 * (on different streams, or from different threads) race on the array. */
fftb_status fftb_sphere_to_grid_static(fftb_plan plan, const void* sphere_in, void* grid_out,
                                       void* stream);

/* Fill *info. Valid for host-only plans too. */
fftb_status fftb_plan_get_info(fftb_plan plan, fftb_plan_info* info);

/* Bytes of device memory the plan holds (tables + scratch). */
fftb_status fftb_plan_workspace_size(fftb_plan plan, size_t* bytes);

/* Per-sphere table summary: occupied columns and occupied x planes. */
fftb_status fftb_plan_sphere_stats(fftb_plan plan, int32_t sphere, int32_t* ncolumns,
                                   int32_t* nslab);

/* Copy the column table of one sphere to host arrays (testing and tools):
 * col_x, col_y: ncolumns entries each (grid x and y of each column, in the
 * plan's column order); entry_col, entry_z: Ns entries each (the column and
 * the z of coefficient g). Any pointer may be NULL to skip that array. */
fftb_status fftb_plan_sphere_columns(fftb_plan plan, int32_t sphere, int32_t* col_x,
                                     int32_t* col_y, int32_t* entry_col, int32_t* entry_z);

/* Per-kernel timing of execute calls, measured with HIP events recorded on
 * the execute stream around each kernel launch (not available for graph
 * replays). Index 0: column kernel, inverse; 1: plane kernel, inverse;
 * 2: plane kernel, forward; 3: column kernel, forward; 4: class combine,
 * forward (plans whose forward plane kernel writes class partials). */
typedef struct {
  int64_t launches[5];
  double total_ms[5];
} fftb_profile;

/* Turn per-kernel event timing on (enable != 0) or off for later execute calls. */
fftb_status fftb_plan_set_profiling(fftb_plan plan, int32_t enable);

/* Wait for the recorded events, return the accumulated launches and
 * milliseconds since the previous call, and reset the accumulators. */
fftb_status fftb_plan_get_profile(fftb_plan plan, fftb_profile* out);

/* Destroy the plan and free its device memory. NULL is accepted. */
fftb_status fftb_plan_destroy(fftb_plan plan);

/* Static description of a status code. */
const char* fftb_status_string(fftb_status status);

/* Thread-local detail of the last failure on this thread ("" if none). */
const char* fftb_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FFTB_H */

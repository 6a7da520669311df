// Kernel argument block shared by the host launcher and the HIP kernels.
#pragma once

#include <cstdint>

namespace fftb {

constexpr int kAxisStages = 8;

// Inverse class pairs: (slab, band) lines per thread whose second class waits
// in registers; the plane kernel and the host's overflow sizing both use it.
template <typename T>
constexpr int kPairRegLines = sizeof(T) == 4 ? 2 : 1;

// Row stride, in 16-byte entries, of the band-inner lines' LDS twiddle table
// (one row of E twiddles per line position): odd, so that the rows a wave
// reads at once start in different LDS banks (rows of 16 entries, 256 bytes,
// all began in the same banks). The kernels and the host's LDS sizing both
// use it.
constexpr int tw_row_stride(int e) { return e | 1; }

struct AxisDev {
  int n;
  int nst;
  int R[kAxisStages];
  int p[kAxisStages];
  int twoff[kAxisStages];
};

// Per-sphere descriptor (device resident). Offsets are in complex elements
// (data buffers) or int32 entries (tables).
struct SphereDesc {
  int64_t sph_off;     // first S[g][b] of this sphere in the sphere buffer
  int64_t grid_off;    // first G[z][y][x][b] in the grid buffer
  int64_t col_off;     // first element of this sphere's column scratch
  int64_t zp_off;      // first element of this sphere's forward class partials
  int32_t gidx_off;    // ncol*nz table: coefficient index of (column, z) or -1
  int32_t colidx_off;  // nslab*ny table: scratch slot of the column at (slab, y) or -1
  int32_t colmeta_off; // per-column slab index, y and scratch slot
  int32_t xinv_off;    // nx table: slab index of x or -1
  int32_t ncol;
  int32_t npcol;       // scratch slots per plane (>= ncol: zero-padded y blocks)
  int32_t nslab;
  int32_t nb;
  int32_t nchunk;      // ceil(nb / band_chunk)
  int32_t nchunk2;     // the same for the band chunk of the plane kernel (band-inner lines)
  int32_t nbp;         // element stride between the band vectors of the column scratch and the
                       // class partials: nchunk*band_chunk, plus one 128-byte line when that
                       // is a multiple of 256 bytes (keeps strided runs off one L2 channel)
  int32_t k1_start, k1_end;  // task range of the column kernel
  int32_t k2_start, k2_end;  // task range of the plane kernel
  int32_t k3_start, k3_end;  // task range of the forward class combine
  int32_t slab_off;    // nslab+1 table: first column of each occupied slab
  int32_t split_off;   // nsplit+1 table: first slab of each forward column split
  int32_t sl_off;      // first slab of this sphere in the per-slab tables
};

struct KArgs {
  int nx, ny, nz;
  int bcl;           // log2(band chunk)
  int bcl2;          // log2(band chunk) of the band-inner plane kernel (may be narrower)
  int n1, m;         // y residue classes and class length m = ny / n1
  int lx;            // rows per x batch in the plane kernel
  int lc;            // columns per column-kernel task
  int nsph;
  int k1_tasks, k2_tasks, k3_tasks;
  int persistent;
  int lds_P, lds_X0, lds_X1;  // element offsets of LDS regions (S starts at 0)
  int lds_acc;       // element offset of the forward column accumulators
  int lds_tab;       // byte offset of the inverse fold's block lists and roots
  int lds_twx;       // byte offset of the band-inner x twiddle table (plane kernel)
  int zline;         // element offset of the spare class-slab line (band-inner x lines)
  int acc_lds;       // forward plane kernel accumulates columns in LDS
  int sx;            // element stride between slab lines of the class slab
  int nsplit;        // forward plane tasks per (plane, chunk): slab ranges with their columns
  int fwd_cls;       // forward: class partials Z[z][xi][j][r], combined into columns by K3
  int g2;            // plane-kernel tasks per L2-sharing group (scheduling)
  int plane32;       // every per-plane region (grid plane, column plane, class
                     // partials of a plane) spans less than 2 GiB
  int k1buf;         // every sphere's coefficients and column region span less than 4 GiB
  int qc;            // inverse band-inner plane tasks: y classes per task (1, or 2: r and r + n1/2)
  int mfma;          // band-inner plane kernel: length-16 fold transforms on the matrix cores
  int ovf_lines;     // class pairs: lines per task whose second class waits in the overflow scratch
  int64_t ovf_off;   // class pairs: element offset of the overflow scratch in the column scratch
  AxisDev ax, ay, az;
  const SphereDesc* sph;
  const int32_t* gidx;
  const int32_t* colidx;
  const int32_t* col_xi;
  const int32_t* col_y;
  const int32_t* xinv;
  const int32_t* slabstart;
  const int32_t* splits;
  const int32_t* col_slot;   // per column: scratch slot
  const int32_t* slab_blk;   // per sphere nslab*n1 (inverse n1): the slab's y blocks that hold
                             // columns, as (first slot << 10 | block index), ascending
  const int32_t* slab_nblk;  // per slab: number of such blocks
  const int32_t* slab_order; // per sphere: slab indices by descending column count
  const void* twx;      // forward-sign twiddles (double pairs, or FP32 hi)
  const void* twy;
  const void* twz;
  const void* twf;      // exp(-2*pi*i*j/ny), j < ny (fold twiddles)
  const void* twx_lo;   // FP32 lo parts (null for FP64)
  const void* twy_lo;
  const void* twz_lo;
  const void* twf_lo;
  const void* rootx;    // exp(-2*pi*i*j/nx), j < nx (register path)
  const void* rootx_lo;
  const void* rootz;    // exp(-2*pi*i*j/nz), j < nz
  const void* rootz_lo;
  const void* in;
  void* out;
  const void* pot;      // inverse: real potential V[z][y][x] multiplied into the grid, or null
  void* col;            // column scratch
  double scale;         // 1/N for the forward direction
  unsigned int* counters;  // 24 work counters (persistent mode): 8 per kernel
};

}  // namespace fftb

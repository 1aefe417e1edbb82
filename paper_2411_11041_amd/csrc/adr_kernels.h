// Device-side argument blocks and kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

namespace adr {

// Line data of one family (all instances concatenated).
template <typename T>
struct LineArgs {
    const int *loff;     // first node of line
    const int *lcnt;     // nodes of line (including the two Dirichlet ends)
    const int *linst;    // instance of line
    const int *inst_nx;  // blocked row stride per instance, 32 ceil(nx / 8)
    const int *cell;     // per node: blocked index of the bottom-left cell corner (-1 at ends)
    const T *lx, *ly;    // per node: offsets in the cell (eq. (23))
    const T *h;          // per node: chord to the previous node
    const T *w;          // per node: |beta| (beta family only)
    const T *L;          // per node: load int f phi (beta family only)
    const int *lidx;     // optional: the line at each list position (active lines only), else line = position
    int lbase;           // list position of the launch's first workgroup (length buckets)
    const T *gend;       // optional: per line the Dirichlet values at its two ends (2 per line); NULL: zero
    int *sing;           // optional: per instance, set to 1 when a pivot is not finite or below ptol
    double ptol;         // relative pivot threshold (of |diagonal| + |eliminated part|)
    const T *phi;        // optional (beta family): per node, phi(Pe) = Pe coth(Pe) of the element
                         // ending at the node, the scale of its exponentially fitted stiffness;
                         // NULL: plain Galerkin rows
    // interpolation-free transfer: when dk is set the node values
    // come from the other family's line values fin instead of the bilinear
    // gather: node k takes (dk[k].x >= 0 ? dw[4k] fin[dk.x] + dw[4k+1] fin[dk.x+1] : dw[4k] x_first)
    // + (dk[k].y >= 0 ? dw[4k+2] fin[dk.y] + dw[4k+3] fin[dk.y+1] : dw[4k+2] x_last)
    const int2 *dk;
    const T *dw;         // FP64 sweeps
    // FP32 sweeps: the same records in 10 bytes (kDir* codes below): dk0 the
    // left bracket's source node (the right one's when the left is the curve's
    // end, or -1 when both are), dkd the right one's offset from dk0 or a code,
    // dwp the left bracket's weight wL (bits 0-9, a fraction of 1023) and the
    // positions tL, tR on the two source segments (bits 10-20, 21-31, fractions
    // of 2047): weights wL(1 - tL), wL tL, wR(1 - tR), wR tR with wR = 1 - wL
    const int *dk0;
    const short *dkd;
    const unsigned *dwp;
    double *lpart;       // optional with dk: per line, sum over its interior nodes of
                         // (new value - old value in vout)^2, at lpart[lslot[line]]
    const int *lslot;
    float *dout;         // optional with dk: per node, new value - old value in vout (0 at the ends)
    double *vacc;        // optional with dk: per interior node, vacc += new value
    float *vacc32;       // optional with dk: the same into an FP32 sum
    // optional (k_line, the one launch per family): XCD-dealt dispatch.
    // Workgroup w runs on XCD w mod 8 as its (w div 8)-th; XCD x takes the list
    // positions xs[x] .. xs[x+1]-1 (through lidx) in order, and workgroups
    // beyond them exit at once.  The set-up deals chunks of neighbouring
    // curves to the XCDs in turn, so that the curves one XCD solves at a time
    // read neighbouring data through its L2, and every XCD gets a share of
    // long and short curves
    const int *xs;
};

// Line launches deal their list to the 8 XCDs in chunks of this many
// neighbouring curves, chunk c to XCD c mod 8 (measured on C2 2049^2: 16 and
// 32 best, 8 and 64 slower)
constexpr int kXcdChunk = 32;

// Codes of LineArgs::dkd: no left bracket on a source segment (the right one
// is dk0), no right one, or a right one too far from dk0 (read dk[k].y)
constexpr short kDirNoLeft = -32766;
constexpr short kDirNoRight = -32767;
constexpr short kDirEscape = -32768;
constexpr int kDirMaxDelta = 32765;

// Record indices relative to the slot's first record (ScatterArgs::rd)
constexpr short kRecMissing = -32768;  // no record
constexpr short kRecEscape = -32767;   // too far from the first: read rk
constexpr int kRecMaxDelta = 32766;

// Scatter stencils of one family; slot s < npad (padded per instance to 256).
// The 4 records of a slot reference nearby line nodes, so they are stored as
// the first record's node (rk0) and three 16-bit offsets from it (rd); a
// record too far away (or whose first record is missing) is marked
// kRecEscape and read from the full table rk.
template <typename T>
struct ScatterArgs {
    const int *gidx;      // blocked index of the interior node, -1 for padding
    const int *blk_inst;  // instance of each 256-slot block
    const int *rk;        // [4][npad] first node of the record's segment, -1 unused (escapes only)
    const int *rk0;       // [npad] rk[0]
    const short *rd;      // [3][npad] rk[r] - rk0 for r = 1..3, or kRecMissing / kRecEscape
    // the weights of v[k] and v[k+1] factored: ca_r = W_r lam_r (1 - t_r), cb_r = W_r lam_r t_r
    // (records 0, 1 take W_h and lam_h, 1 - lam_h; records 2, 3 W_v = 1 - W_h and lam_v, 1 - lam_v)
    const unsigned *sw;   // [npad] bits 0-1: 2 W_h; FP32 sweeps: bits 2-16 lam_h, 17-31 lam_v (15-bit
                          // fractions)
    const unsigned *rt;   // FP32 sweeps: [2][npad] t of records 0, 1 (then 2, 3) as 16-bit fractions,
                          // low half first
    const double *rf;     // FP64 sweeps: [6][npad] lam_h, lam_v, t_0 .. t_3
    int npad;
    const int *blist;     // optional: the slot block of each workgroup (active blocks only)
    int nblist;           // workgroups when blist is set
    const double *gb;     // optional ([npad], FP64 sweeps of the state only): the boundary points'
                          // share of the Dirichlet data in the slot's value; NULL: zero data
};

// The grid fields the sweeps use (state, half step, increments) are stored in
// blocks of 8 x 4 nodes (one 128-byte line in FP32): node (x, y) of an
// instance sits at
//   boff + ((y / 4) * nx8 + x / 8) * 32 + (y % 4) * 8 + x % 8,   nx8 = ceil(nx / 8),
// with boff a multiple of 32, so that the corner gathers of a curve touch few
// cache lines whatever its direction.  The caller's arrays stay row-major.
__host__ __device__ inline int blocked_index(int x, int y, int boff, int bstride) {
    return boff + (y >> 2) * bstride + ((x >> 3) << 5) + ((y & 3) << 3) + (x & 7);
}

// dynamic LDS of the line solve of family fam (0 beta, 1 gamma) whose longest curve has nmax nodes
template <typename T>
size_t line_lds_bytes(int fam, int nmax);

// Length buckets of the line solve: curves of at most 12, 8, 4, 2, 1 nodes per
// thread (bucket 0..4); a curve of `nodes` nodes belongs to line_bucket(nodes).
constexpr int kLineBuckets = 5;
int line_bucket(int nodes);

// Workgroup shapes of bucket b (rows per thread x threads per curve): shape
// 0 .. line_shapes(b) - 1, shape 0 the default.
int line_shapes(int bucket);

// bucket -1: one launch for curves of any length (a register footprint per
// workgroup inside the kernel; shape ignored); bucket b: every curve of the
// launch lies in b and is solved with the given shape.  n_lines workgroups
// take the list positions a.lbase .. a.lbase + n_lines - 1; with a.xs (bucket
// -1 only) n_lines is the grid, 8 times the longest XCD share.
template <typename T>
hipError_t launch_line(int fam, int bucket, int shape, const LineArgs<T> &a, int n_lines, const T *fin, T *vout,
                       const double *par, const int *done, int nmax, hipStream_t st);

// interior nodes between the caller's row-major array and the blocked layout:
// to_blocked: blk[gb[s]] = rm[gr[s]]; otherwise rm[gr[s]] = blk[gb[s]] (slots s < npad, gr < 0: padding)
hipError_t launch_layout(const int *gr, const int *gb, int npad, const double *src, double *dst, bool to_blocked,
                         hipStream_t st);

template <typename T, typename TO>
hipError_t launch_scatter(int mode, const ScatterArgs<T> &s, const T *v, TO *out, float *d32, double *partial,
                          const int *done, hipStream_t st);

hipError_t launch_norm(int n_inst, const double *partial, const int *blk_start, double *cnorm, double *rel, int *done,
                       int *it_count, int count, double tol, int mode, hipStream_t st);

hipError_t launch_fill_int(int *p, int v, int n, hipStream_t st);

// ---- GMRES acceleration: per-instance vector operations on FP64 blocked fields
// Each instance's blocked range is cut into chunks of krylov_chunk() entries.
struct KChunks {
    const int *inst;            // [n] instance of each chunk
    const int64_t *begin, *end;  // [n] entry range of each chunk
    const int *inst_chunk;      // [n_inst + 1] first chunk of each instance
    int n, n_inst;
};
int krylov_chunk();
// out[i * kmax + v] = (z, V_v) per instance i, v < nv (V_v at V + v * stride); partial: [n][kmax]
hipError_t launch_kdot(const double *z, const double *V, int64_t stride, int nv, int kmax, const KChunks &ch,
                       const int *done, double *partial, double *out, hipStream_t st);
// z <- V_j - z - sum_{v < nv} coef[i * kmax + v] V_v; out[i * kmax] = |z|^2 per instance
hipError_t launch_kupdate(double *z, const double *V, int64_t stride, int j, int nv, int kmax, const double *coef,
                          const KChunks &ch, const int *done, double *partial, double *out, hipStream_t st);
// x += sum_{v < nv} coef[i * kmax + v] V_v
hipError_t launch_kcombine(double *x, const double *V, int64_t stride, int nv, int kmax, const double *coef,
                           const KChunks &ch, const int *done, hipStream_t st);
// v *= scale[i * kmax]
hipError_t launch_kscale(double *v, const double *scale, int kmax, const KChunks &ch, const int *done,
                         hipStream_t st);
// r = phi - u on the interior nodes (gb: blocked index of each scatter slot, -1 padding)
hipError_t launch_kresidual(const int *gb, int npad, const double *phi, const double *u, double *r, hipStream_t st);

// v on the curve nodes of a's family: the Dirichlet values at the ends (a.gend,
// or zero) and on the interior nodes the bilinear gather of U (eq. (22)), or
// zero when U is NULL.  One workgroup per curve of the full list.
hipError_t launch_line_values(const LineArgs<double> &a, int n_lines, const double *U, double *v, hipStream_t st);
// the same from an FP32 blocked field into FP32 curve values (ends from a.gend,
// NULL for increments), clearing zacc (when set) on the same nodes; the lines
// are a.lidx[0 .. n_lines) when a.lidx is set
hipError_t launch_line_values32(const LineArgs<float> &a, int n_lines, const float *U, float *v, float *zacc,
                                hipStream_t st);

// Lout = Lbase + M G un / dt on the interior nodes of the beta-curves (the
// full line list of a), ends copied: the load of an implicit Euler step.
hipError_t launch_shift_load(const LineArgs<double> &a, int n_lines, int nmax, const double *Lbase, const double *un,
                             double *Lout, double inv_dt, hipStream_t st);

// Order-preserving compaction of the items (lines or slot blocks) whose
// instance inst_of[i] is not done: idx receives their indices, *count (device)
// their number.  bcnt: scratch of ceil(n / 256) + 1 ints.
hipError_t launch_compact(const int *inst_of, int n, const int *done, int *bcnt, int *idx, int *count, hipStream_t st);

}  // namespace adr

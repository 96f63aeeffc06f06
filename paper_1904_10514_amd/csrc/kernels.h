// Device kernels of libhp2sph and their launch wrappers (gfx950, wave64).
//
// Data layout shared by the stages (one nside group of `nmaps` maps):
//   Dsym_b [h][n]   block b = 0..3 (see tables.h), h = 0 .. 2 nside (the pole
//                   row, the ring pairs, the equator), n = column of
//                   (map, k', c) (GroupDims::cm/ck) with k' = k / 2 the index
//                   of the longitude mode k of the block's parity and c = 0
//                   (real), 1 (imaginary).
//   U_b    [l'][n]  order-0/1 Legendre coefficients of block b (after the
//                   fused colatitude fit), then, in place, a_l^m after the
//                   Givens sweeps: column k' holds order m = 2k' + kpar at
//                   degrees l = lmin + 2 l' >= m.
// Every array is row-major with the row stride N_kpar = nmaps * Npm_kpar,
// Npm_kpar = 2 * (number of modes of parity kpar).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <vector>

namespace hp2sph {

template <class T>
struct FftTab {
    const T* twiddle;         // e^{-2 pi i t / fft_max}, t < fft_max (complex)
    const T* roots;           // per ring size: e^{-i pi k / n}, k = 0 .. n
    const T* chirp;           // per ring size (Bluestein): w_k = e^{-i pi k^2 / L}
    const T* chirpfft;        // per ring size (Bluestein): FFT_M(conj chirp)
    const int64_t* rootoff;   // [j], j = 1 .. nside (complex offsets)
    const int64_t* chirpoff;
    const int64_t* chirpfftoff;
    const int32_t* chirpm;    // Bluestein length per j, 0 if L = 2j is a power of two
    int fft_max;
};

struct RingTab {
    const int64_t* start;     // first pixel of ring r (index r - 1)
    const int32_t* n;         // pixels on ring r
    const int8_t* shifted;    // 1 if the first point is at pi / n, 0 if at 0
};

template <class T>
struct Blocks4 {
    T* p[4];
};

struct GroupDims {
    int nside, p, nmaps;
    int Npm[2];               // columns per map for k parity 0 / 1
    int64_t N[2];             // row strides nmaps * Npm
    int nl[4], nk[4], lmin[4], tpad[4];
    // column of (map, k', c) within a row: map * cm[kpar] + k' * ck[kpar] + c.
    // map-major (staged strategy; the sweeps need k' contiguous): cm = Npm,
    // ck = 2.  mode-major (tables strategy; one mode's maps contiguous for the
    // per-order GEMMs): cm = 2, ck = 2 * nmaps.
    int64_t cm[2], ck[2];
    int modemajor;
};

// Workspace regions of one nside group (Dsym- or U-shaped, four blocks each):
// D (Dsym; the synthesis GEMM output in the refinement), U (order-0/1 or
// a_l^m coefficients; the FP64 a0 and then the FP32 correction in the
// refinement), Df (FP64 ring coefficients of the maps), Dr (FP32 residual
// coefficients), Ua (FP32 a0).  Every group of a plan has its own regions,
// so that one launch can serve all groups.
enum Region { kRegD = 0, kRegU = 1, kRegDf = 2, kRegDr = 3, kRegUa = 4, kRegions = 5 };

// Everything the work-list kernels need of one group, in device memory (one
// array per plan).  reg[r][b]: byte offset of block b of region r from the
// workspace base (-1: the plan has no such region).
struct GroupDesc {
    GroupDims g;
    RingTab rt;
    FftTab<double> ft;
    const int64_t* map_off;     // per member: first pixel of its map
    const int64_t* alm_off;     // per member: first alm entry (complex)
    const int32_t* lmax;        // per member
    const int32_t* pack_tiles;  // (m, l0) of the pack tiles
    int n_pack_tiles;
    int tables;                 // per-order tables (mode-major columns)
    double pole_w[3];
    int64_t reg[kRegions][4];
};

// A work-list launch over groups first .. first + n - 1 of a plan's
// GroupDesc array: group first + i owns work items [start[i], start[i] +
// count[i]); every start is a multiple of 8, so an item's index modulo 8 is
// the XCD the hardware deals its workgroup to (items past count are padding
// and do nothing).  A launch of fewer workgroups than items (persistent)
// walks the list with a stride of its grid size, a multiple of 8.
constexpr int kMaxGroups = 16;
struct GroupRange {
    int first, n;
    int32_t start[kMaxGroups + 1];
    int32_t count[kMaxGroups];
};

// Host side of a work-list launch: the device descriptors, their host
// copies (for the item counts), the group span, the workspace, the grid
// cap (0: one workgroup per item; else the persistent grid size) and the
// kernel variant where a stage has several (the pack's maps per tile: 16,
// 32 or 64; the ring transform's item order 0, 1 or 2; 0 for the default).
struct GroupLaunch {
    const GroupDesc* dev;
    const GroupDesc* host;
    int first, n;
    char* ws;
    int grid_cap;
    int variant;
    int threads = 0;   // ring transform: 512 runs nside <= 1024 with 512 threads (8 values each)
};

// One product of a grouped GEMM: C[m][n] = sum_k A[k][m] B[k][n].
// A is absolute (a set-up table); B and C are element offsets from the
// launch's base pointers, so a problem list can be built once per plan and
// reused with any workspace.  Column n of B (C) is at (n >> 1) * bps + (n & 1)
// (pair stride; 2 = contiguous), which lets a problem pick one mode's
// (re, im) pair out of every map of an interleaved layout.
template <class T>
struct GemmProblem {
    const T* A;               // [K][M], row stride lda
    int64_t boff, coff;       // element offsets of B and C
    int M, N, K;
    int64_t lda, ldb, ldc;
    int64_t bps, cps;         // column-pair strides of B and C
    int tiles_n, tile_begin;  // set by finalize_gemm_problems
};

// Row stride of a per-order analysis table with M columns: padded to a
// multiple of 4 elements so that its rows can be read as 16-byte vectors.
__host__ __device__ inline int order_table_lda(int M) { return (M + 3) & ~3; }

// Staging geometry of the grouped GEMM (128 x 128 output tiles, k steps of 16
// rows, 256 threads), shared by the kernel and the host-side replay of its
// addresses.  Thread tid stages 8 elements of k row tid / 16 of each operand
// tile: its 16-byte vector q sits at column 16 VE q + VE (tid % 16), VE the
// elements per 16 bytes, so the 16 lanes of a row cover one contiguous run.
// The staging loads are raw buffer loads: per k step one descriptor for A
// and one for B span the step's rows that lie in the problem, and an element
// outside the problem's columns gets the offset kGemmOOB, past every
// descriptor, so the hardware returns zero for it.
constexpr int kGemmBM = 128, kGemmBN = 128, kGemmBK = 16, kGemmThreads = 256;
constexpr uint32_t kGemmOOB = 0x80000000u;
template <class T>
struct GemmStage {
    static constexpr int VE = 16 / int(sizeof(T));   // elements per 16-byte vector
    // k row (within the step) and column (within the tile) of element e of thread tid
    __host__ __device__ static int row(int tid) { return tid >> 4; }
    __host__ __device__ static int col(int tid, int e) { return (tid & 15) * VE + (e / VE) * (16 * VE) + (e % VE); }
};
// Rows of the k step that starts at k0 (k0 < K).
template <class T>
__host__ __device__ inline int gemm_step_rows(const GemmProblem<T>& P, int k0) {
    return P.K - k0 < kGemmBK ? P.K - k0 : kGemmBK;
}
// A is read as 16-byte vectors when its row stride and base allow it; the
// vector at column mm then covers mm .. mm + VE - 1 < lda (the row padding).
template <class T>
__host__ __device__ inline bool gemm_a_vector(const GemmProblem<T>& P) {
    return (P.lda % GemmStage<T>::VE) == 0 && (reinterpret_cast<uintptr_t>(P.A) % 16) == 0;
}
// Bytes covered by the A / B descriptors of the k step at k0 (their bases are
// A + k0 lda and B + k0 ldb): every row of the step up to the end of the
// problem's elements in its last row, so that a descriptor never reaches past
// the operand (a problem's columns may start inside a row of a wider array).
// The vector loads of A read up to the row padding (column lda).
// A problem with K = 0 (a synthesis order with no degree: its output is zero)
// still stages one step, of no rows: its descriptors are empty.
template <class T>
__host__ __device__ inline uint32_t gemm_a_records(const GemmProblem<T>& P, int k0) {
    const int rows = gemm_step_rows(P, k0);
    if (rows <= 0) return 0;
    const int64_t last = gemm_a_vector(P) ? P.lda : P.M;
    return uint32_t((int64_t(rows - 1) * P.lda + last) * int64_t(sizeof(T)));
}
template <class T, class TB>
__host__ __device__ inline uint32_t gemm_b_records(const GemmProblem<T>& P, int k0) {
    const int rows = gemm_step_rows(P, k0);
    if (rows <= 0) return 0;
    return uint32_t((int64_t(rows - 1) * P.ldb + int64_t((P.N - 1) >> 1) * P.bps + 2) * int64_t(sizeof(TB)));
}
// Byte offset of the A load of element e (a 16-byte vector at e % VE == 0 when
// gemm_a_vector, else one element) of thread tid in the tile at row m0.
template <class T>
__host__ __device__ inline uint32_t gemm_a_offset(const GemmProblem<T>& P, bool avec, int m0, int tid, int e) {
    const int mm = m0 + GemmStage<T>::col(tid, e);
    const bool in = avec ? mm < P.lda : mm < P.M;
    return in ? uint32_t((GemmStage<T>::row(tid) * int(P.lda) + mm) * int(sizeof(T))) : kGemmOOB;
}
// Byte offset of the (re, im) pair load of elements e, e + 1 (e even) of B in
// the tile at column n0.
template <class T, class TB>
__host__ __device__ inline uint32_t gemm_b_offset(const GemmProblem<T>& P, int n0, int tid, int e) {
    const int nn = n0 + GemmStage<T>::col(tid, e);
    return nn < P.N ? uint32_t((GemmStage<T>::row(tid) * int(P.ldb) + (nn >> 1) * int(P.bps)) * int(sizeof(TB)))
                    : kGemmOOB;
}

// Assign tile ranges (in list order) and return the number of tiles.
template <class T>
int finalize_gemm_problems(GemmProblem<T>* p, int n);

// Workgroup -> (problem, tile) map that keeps every problem on one XCD:
// problems are dealt to the 8 XCDs in list order (longest first), and
// workgroup id is placed so that id mod 8 (the XCD the hardware dispatches it
// to) is the problem's XCD.  Entries of -1 pad the XCDs to equal length.
template <class T>
std::vector<int32_t> xcd_tile_map(const GemmProblem<T>* p, int n);

// Threads of the ring kernels for a plan whose largest FFT has fft_max points
// (at most 16 complex values per thread).
__host__ __device__ constexpr int ring_threads(int fft_max) { return fft_max <= 4096 ? 256 : 512; }

// S1: per-ring real DFT, shift to unshifted longitudes, Nyquist rule and the
// north/south combination, written into Dsym rows 1 .. 2 nside of region
// `reg` of every group of the launch (FP64).  Work item: (map, ring pair), in
// the order gl.variant selects (0: XCD-aware, 1: pair-major, 2: map-major).
hipError_t launch_ring_forward(const double* maps, const GroupLaunch& gl, int reg, hipStream_t s);

// Equal-weight analysis, eq. (healsph): longitude sums of every ring for all
// modes m = 0..p (aliased beyond each ring's Nyquist mode), combined per ring
// pair as W+- = scale (F_N +- F_S) into Dsym rows 1 .. 2 nside (row 0 is not
// written).
hipError_t launch_ring_adjoint(const double* maps, const int64_t* map_off, RingTab rt, FftTab<double> ft,
                               Blocks4<double> W, const GroupDims& g, double scale, hipStream_t s);

// Equal-weight iteration: Wr = Wf - W(S a) for Dsym rows 1 .. 2 nside, with
// W(S a) the weighted longitude sums (as launch_ring_adjoint writes them) of
// the rings synthesized from the synthesis GEMM output Gs, formed from the
// coefficients by alias-chain sums (no transform).
hipError_t launch_adjoint_residual(Blocks4<const double> Wf, Blocks4<const double> Gs, Blocks4<double> Wr, RingTab rt,
                                   const GroupDims& g, double scale, hipStream_t s);

// Refinement residual in ring-Fourier space: Dr = Df - Ring(Synth(Gs)) for
// Dsym rows 1 .. 2 nside (Gs: synthesis GEMM output in region D, Df: FP64
// forward ring coefficients of the maps), written in FP32 to region Dr.
// Work item: (16 maps, ring pair).
hipError_t launch_residual_fold(const GroupLaunch& gl, hipStream_t s);

// S2: pole row h = 0 of region `reg` (quadratic extrapolation of the three
// nearest ring means); zeroes every other entry of the pole row.
template <class T>
hipError_t launch_pole(const GroupLaunch& gl, int reg, hipStream_t s);

// Grouped GEMM over a device-resident problem list (finalized), one launch.
// B is stored as TB (offsets boff in TB elements) and rounded to T.
template <class T, class TB = T>
hipError_t launch_gemm(const GemmProblem<T>* probs_dev, const int32_t* tmap_dev, int nslots, const TB* Bbase,
                       T* Cbase, hipStream_t s);

// Set-up helpers for the per-order tables (see api.cpp):
// U_v[l'][(v, k', c)] = M[row(h)][l'] (or M[l'][h]) for h = h_first + 2v + c,
// replicated over every column k' of the block.
template <class T>
hipError_t launch_replicate(const T* mat, int64_t rs, int64_t cs, int nl, int h_first, int h_last, T* Uv, int nk,
                            int nv, hipStream_t s);
// Copy finished columns out of U_v into per-order tables.
//   analysis:  tab[off[k']] [h - h0(k')][l' - k']   for h >= h0(k'), l' >= k'
//   synthesis: tab[off[k']] [l' - k'][h - 1]        for h >= 1,      l' >= k'
template <class T>
hipError_t launch_scatter_tables(const T* Uv, int nl, int nk, int nv, int h_first, int h_last,
                                 const int64_t* off, const int32_t* h0, int ldm_syn, bool synthesis, T* tab,
                                 hipStream_t s);
hipError_t launch_convert(const double* in, float* out, int64_t n, hipStream_t s);
// Per-order adjoint tables: adj[aoff[k']][h][l] = syn[soff[k']][l][h], h < H,
// l < nl - k', adjoint row stride order_table_lda(nl - k') (padding untouched).
hipError_t launch_transpose_orders(const double* syn, const int64_t* soff, double* adj, const int64_t* aoff, int nl,
                                   int nk, int H, hipStream_t s);

// S4 analysis sweeps (Givens, order 0/1 -> order m), in place on U.
template <class T>
hipError_t launch_sweep_fwd(Blocks4<T> U, Blocks4<const T> G, const GroupDims& g, hipStream_t s);

// Synthesis sweeps (transposed, order m -> order 0/1), in place on U.
template <class T>
hipError_t launch_sweep_bwd(Blocks4<T> U, Blocks4<const T> G, const GroupDims& g, hipStream_t s);

// U (a_l^m after the sweeps, region reg_a) -> packed complex128 alm; with
// reg_b >= 0 writes Ua + Ub (added in FP64).  Work item: (order m, 64 l, 32
// maps), the group's pack tiles.
template <class T>
hipError_t launch_pack(const GroupLaunch& gl, int reg_a, int reg_b, double* alm, hipStream_t s);
// (m, l0) of every pack tile of the mode-major layout (per-order tables):
// orders m = 0..p, l0 = m, m + 64, ... <= p.
std::vector<int32_t> pack_tiles(int p);
// (m0, l0) of every pack tile of the map-major layout (staged strategy): 16
// orders m0, m0 + 2, .. of one parity, l0 = m0, m0 + 64, ... <= p.
std::vector<int32_t> pack_tiles_mapmajor(int p);

// FP32 U (region Ua) -> FP64 U (region U) in the same layout, zero outside
// m <= l <= lmax(map); groups with per-order tables leave the rows l < m
// (never read by their GEMMs) unwritten.
hipError_t launch_widen(const GroupLaunch& gl, hipStream_t s);

// Jacobi update in the U layout of per-order tables (mode-major only):
// Uacc = (first ? 0 : Uacc) + U for m <= l <= lmax(map), zero above lmax,
// rows l < m untouched.
hipError_t launch_accumulate(Blocks4<const double> U, Blocks4<double> Uacc, const int32_t* lmax, const GroupDims& g,
                             bool first, hipStream_t s);

// packed complex128 alm -> U (zeros outside 0 <= m <= l <= lmax).
hipError_t launch_unpack(const double* alm, const int64_t* alm_off, const int32_t* lmax, Blocks4<double> U,
                         const GroupDims& g, hipStream_t s);

// Synthesis: Dsym (FP64, from the evaluation GEMM) -> ring values; if
// `minus_from` is non-null writes minus_from - synthesis (the residual).
hipError_t launch_ring_inverse(Blocks4<const double> D, RingTab rt, FftTab<double> ft, double* out,
                               const double* minus_from, const int64_t* map_off, const GroupDims& g,
                               hipStream_t s);

// Raise the dynamic-LDS limit of the ring kernels (up to 139 KB at nside 2048).
hipError_t configure_kernels();

// Size of the static device workspace of the allocation-free analysis
// (HP2SPH_NOALLOC_WORKSPACE of the C ABI).
constexpr size_t kScratchBytes = size_t(256) << 20;
// Looks up (once per device, with that device current) the device address of
// the static workspace; scratch_ptr(device) returns it afterwards (null if
// scratch_init never ran on that device).
hipError_t scratch_init();
void* scratch_ptr(int device);

// C_l per map from packed alm.
hipError_t launch_cl(const double* alm, const int64_t* alm_off, const int32_t* lmax, double* cl,
                     const int64_t* cl_off, int nmaps, int lmax_max, hipStream_t s);

}  // namespace hp2sph

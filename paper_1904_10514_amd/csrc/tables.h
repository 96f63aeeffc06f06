// Host-side set-up tables for one nside (FP64), built once per plan.
//
// Geometry of the half-ring rows used by every stage: row h = 0 is the north
// pole, rows h = 1 .. 2 nside are the rings r = h (north) paired with the
// mirror rings r = 4 nside - h (south); h = 2 nside is the equator.  For a
// longitude mode k the ring data of a pair enter only through the sums and
// differences D+- = (D_north +- D_south) / 2, and with the colatitude
// least-squares fit (Sec. 3.2.2 of the paper) split by the parity of k and
// of the Legendre degree l, four independent blocks arise:
//   block 0: k even, D+  -> order-0 Legendre coefficients, l = 0, 2, .., p
//   block 1: k even, D-  -> order-0, l = 1, 3, .., p-1
//   block 2: k odd,  D+  -> order-1, l = 1, 3, .., p-1
//   block 3: k odd,  D-  -> order-1, l = 2, 4, .., p
// (l - k even pairs with D+, l - k odd with D-, since
// Y_l^m(pi - theta) = (-1)^{l+m} Y_l^m(theta)).
#pragma once

#include <cstdint>
#include <vector>

namespace hp2sph {

struct BlockShape {
    int kpar;    // parity of the longitude mode k
    int sym;     // 0: D+, 1: D-
    int lmin;    // smallest Legendre degree of the block
    int nl;      // number of degrees l = lmin, lmin + 2, .., <= p
    int nk;      // number of modes k of parity kpar in 0..p
    int nsweep;  // Givens sweeps needed by the highest column of the block
};

BlockShape block_shape(int nside, int block);

struct RingGeom {
    double z, one_minus_z_abs, phi0;
    int64_t n, start;
};

struct HostTables {
    int nside = 0;
    int p = 0;
    std::vector<RingGeom> rings;        // r = 1 .. 4 nside - 1 at index r - 1
    double pole_w[3] = {0, 0, 0};       // f_pole = sum_r w_r * mean(ring r), r = 1..3
    // analysis matrices, [h][l'] with h = 0 .. 2 nside (K = 2 nside + 1 rows)
    std::vector<double> ana[4];
    // synthesis (evaluation) matrices, [l'][h]
    std::vector<double> syn[4];
    // Givens angles, device layout [l'][t-1][2] (t = 1 .. nsweep; (c, s));
    // entries with l' < t are zero
    std::vector<double> givens[4];
    // FFT tables
    int fft_max = 0;                    // largest power-of-two FFT length
    std::vector<double> twiddle;        // e^{-2 pi i t / fft_max}, t < fft_max, (re, im)
    // per ring size n = 4j (j = 1 .. nside): offsets into the tables below
    std::vector<int64_t> rootoff;       // e^{-i pi k / n}, k = 0 .. n (n+1 complex)
    std::vector<double> roots;
    std::vector<int64_t> chirpoff;      // Bluestein chirp w_k = e^{-i pi k^2 / L}, L = n/2
    std::vector<double> chirp;
    std::vector<int64_t> chirpfftoff;   // FFT_M of the conjugate chirp (M = Bluestein length)
    std::vector<int32_t> chirpm;        // M per ring size (0 when L is a power of two)
    std::vector<double> chirpfft;
};

// Builds every table for nside (power of two, >= 2).  Multi-threaded.
void build_tables(int nside, HostTables& t, bool with_fft = true);

// Givens (c, s) of the connection from order mp-2 to order mp at degree l.
void givens_cs(int l, int mp, double* c, double* s);

// Ring geometry of eq. (healpts): 1 <= r <= 4 nside - 1.
RingGeom ring_geom(int nside, int r);

int64_t bluestein_length(int64_t L);

}  // namespace hp2sph

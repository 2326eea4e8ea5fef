// sizes.hpp -- transform lengths n the library is compiled for (one object per size):
// 2^a 3^b (b <= 1; 384, 768 and 1536 make padding to B_3 reach n = 256, 512 and 1024),
// 5 * 2^a and 7 * 2^a.
// The build script reads this list.
#pragma once
#define GS_SIZE_LIST(X) X(8) X(12) X(16) X(20) X(24) X(28) X(32) X(40) X(48) X(56) X(64) X(80) X(96) X(112) X(128) X(160) X(192) X(224) X(256) X(320) X(384) X(512) X(640) X(768) X(1024) X(1536) X(2048)
#define GS_MAX_N_3D 1024

// Grid of the fused pass: persistent (rounds of co-resident blocks looping over pencil
// groups, the per-thread stage twiddles kept in registers across groups) only for 3D
// grids of n = 256; one block per pencil group elsewhere, where the twiddles held across
// groups cost occupancy.  Measured fused-pass times, persistent -> one block per group:
// 256^3 0.275 -> 0.295 ms (dipolar 0.320 -> 0.325); 192^3 0.172 -> 0.158; dipolar 128^3
// 0.051 -> 0.048; 512^3 2.64 -> 2.45; 1024^3 26.2 -> 25.0; 2D 2048^2 0.077 -> 0.059 ms;
// Coulomb 64^3 to 128^3 equal within the spread between runs.
constexpr bool gs_fused_persistent(int d, int n) { return d == 3 && n == 256; }

// Lengths for which the cubic passes are also compiled in tile-shape variants (more or fewer
// rows or pencils per block; the same bits) that the plan autotuner chooses among.
constexpr bool gs_tile_variants(int n) { return n >= 128; }

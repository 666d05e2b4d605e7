// Tile-configuration cost model of the MFMA products, shared by the host
// (single calls, batched graphs, serving) and the device (the batched entry
// point picks each matrix's configurations on the device from its shape):
// the same function and table on both sides give the same choice, so every
// tile is computed the same way whichever path runs it.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

namespace psvt {

constexpr int kNumTiles = 4;

__host__ __device__ inline int tile_bm(int c) { return c == 1 ? 64 : c == 2 ? 128 : c == 3 ? 192 : 256; }

// Largest configuration per operand type (f32, bf16, fp8, split bf16) in
// the persistent batched executor: one kernel holds every tile body it may
// run, and these keep its LDS at two blocks per CU.
constexpr int kPersistMaxTile[4] = {2, 2, 1, 1};

// (efficiency, per-tile overhead in microseconds) per operand type, kind
// (sym = lower-triangle product) and configuration 1..4; force: a forced
// configuration (0 = none); max_tile: the largest configuration considered
// per operand type.
struct TileModelTable {
    float eff[4][2][kNumTiles + 1];
    float overhead_us[4][2][kNumTiles + 1];
    int force;
    int max_tile[4];
};

__host__ __device__ inline int tile_count(int M, int N, int sym, int bm) {
    const int nbm = (M + bm - 1) / bm, nbn = (N + bm - 1) / bm;
    return sym ? nbm * (nbm + 1) / 2 : nbm * nbn;
}

// dense MFMA flop/s of one CU per operand type (split bf16: the useful rate,
// a third of bf16's, since every product takes three)
__host__ __device__ inline double cu_rate(int type) {
    return type == 0 ? 157.3e12 / 256.0 : type == 1 ? 2516.6e12 / 256.0 : type == 2 ? 5033.2e12 / 256.0
                                                                                      : 2516.6e12 / 3.0 / 256.0;
}

// Blocks of configuration c that one CU holds at once (its LDS: 160 KB per
// CU; split bf16 keeps both planes of a k-tile up to 128 x 128).
__host__ __device__ inline int tile_occ(int type, int c) {
    if (c >= 3) return 1;
    if (type == 3) return c == 1 ? 2 : 1;
    return c == 1 ? 4 : 2;
}

// The CU with the most tiles, p, does all their flops on its MFMA units, in
// ceil(p / occ) waves of blocks, each wave paying a start and drain:
//   time ~= p x tile flops / (eff x CU rate) + ceil(p / occ) x overhead
__host__ __device__ inline double model_time_us(const TileModelTable &t, int type, int M, int N, int K, int sym,
                                                int c) {
    const double bm = tile_bm(c);
    const double per_cu = ceil(tile_count(M, N, sym, tile_bm(c)) / 256.0);
    const double waves = ceil(per_cu / tile_occ(type, c));
    const int k = sym ? 1 : 0;
    return per_cu * 1e6 * bm * bm * 2.0 * K / (t.eff[type][k][c] * cu_rate(type)) + waves * t.overhead_us[type][k][c];
}

__host__ __device__ inline int pick_tile(const TileModelTable &t, int type, int M, int N, int K, int sym) {
    const int hi = t.max_tile[type] < kNumTiles ? t.max_tile[type] : kNumTiles;
    if (t.force >= 1 && t.force <= hi) return t.force;
    double best = 1e300;
    int arg = hi < 2 ? hi : 2;
    for (int c = 1; c <= hi; ++c) {
        const double v = model_time_us(t, type, M, N, K, sym, c);
        if (v < best * 0.999) {
            best = v;
            arg = c;
        }
    }
    return arg;
}

}  // namespace psvt

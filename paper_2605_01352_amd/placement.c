/* Rejection-sampled spawn positions of the synthetic scenes (input
 * generation only: no physics or raster arithmetic).  The same draws and the
 * same double-precision arithmetic as the numpy version in scenegen.py,
 * evaluated one try at a time:
 *   draw k of a stream with state `key` is mix64(key + (k + 1) GAMMA)
 *   (SplitMix64, Steele, Lea and Flood 2014), a unit double its top 53 bits;
 *   a try takes three draws: x = (-0.5 + R) + (1 - 2R) ux, the same for y,
 *   z = R + (H - 2R) uz; it is kept when its squared distance to every
 *   earlier body of the env exceeds (R_i + R)^2; after 1000 failed tries of
 *   one body the box height H grows by 0.25 m.
 * Built with -ffp-contract=off so that no product is fused. */
#include <stdint.h>

static const uint64_t GAMMA = 0x9E3779B97F4A7C15ull;

static uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static double unit(uint64_t key, uint64_t k) {
  return (double)(mix64(key + (k + 1) * GAMMA) >> 11) * 0x1.0p-53;
}

/* n_envs envs; env e has counts[e] bodies starting at off[e] (bounding radii
 * R[off[e] ..]), stream state keys[e] and box height H[e].  pos receives
 * 3 doubles per body. */
void place_envs(int64_t n_envs, const int64_t* off, const int64_t* counts, const uint64_t* keys, const double* H0,
                const double* R, double* pos) {
  for (int64_t e = 0; e < n_envs; ++e) {
    const int64_t b0 = off[e];
    double H = H0[e];
    uint64_t ctr = 0;
    for (int64_t k = 0; k < counts[e]; ++k) {
      const double r = R[b0 + k];
      int tries = 0;
      for (;;) {
        const double ux = unit(keys[e], ctr), uy = unit(keys[e], ctr + 1), uz = unit(keys[e], ctr + 2);
        ctr += 3;
        const double cx = (-0.5 + r) + (1.0 - 2.0 * r) * ux;
        const double cy = (-0.5 + r) + (1.0 - 2.0 * r) * uy;
        const double cz = r + (H - 2.0 * r) * uz;
        int ok = 1;
        for (int64_t i = 0; i < k && ok; ++i) {
          const double* p = pos + 3 * (b0 + i);
          const double dx = p[0] - cx, dy = p[1] - cy, dz = p[2] - cz;
          const double d2 = (dx * dx + dy * dy) + dz * dz;
          const double rs = R[b0 + i] + r;
          ok = d2 > rs * rs;
        }
        if (ok) {
          pos[3 * (b0 + k)] = cx;
          pos[3 * (b0 + k) + 1] = cy;
          pos[3 * (b0 + k) + 2] = cz;
          break;
        }
        if (++tries >= 1000) {
          H += 0.25;
          tries = 0;
        }
      }
    }
  }
}

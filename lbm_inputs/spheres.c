/*
 * spheres.c -- seeded random overlapping-sphere packs (input generator).
 *
 * Holds no lattice Boltzmann arithmetic: it only produces solid masks.  Both
 * the oracle side and the GPU side take their porous geometries from here.
 *
 * Random numbers: SplitMix64 (Steele, Lea & Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014): the state advances by the
 * golden-ratio increment and each output is the state passed through the
 * 64-bit finaliser with shifts 30/27/31.
 *
 * Pack: spheres of integer radius r are added one at a time.  A sphere's
 * centre is (cx, cy, cz) with c = (next() >> 32) mod n per axis, in the order
 * x, y, z.  A cell is covered when its minimum-image squared distance to the
 * centre is <= r^2 (periodic box).  After each sphere the porosity
 * (fluid cells / cells) is updated; the pack stops at the first sphere after
 * which it is <= the target.
 */
#include <stdint.h>
#include <stdlib.h>

uint64_t sm_next(uint64_t *state)
{
    uint64_t z = (*state += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

void sm_fill(uint64_t *state, uint64_t *out, long n)
{
    for (long k = 0; k < n; ++k) out[k] = sm_next(state);
}

/* Adds spheres to `solid` (uint8, x fastest) until the porosity is <= target
 * or max_spheres were added.  Returns the number of spheres added; *n_solid
 * holds the solid count on entry and on return. */
long sphere_pack(uint8_t *solid, int nx, int ny, int nz, int radius, double target_porosity,
                 uint64_t *state, long max_spheres, long *n_solid)
{
    const long ncell = (long)nx * ny * nz;
    const int r = radius;
    /* ball offsets */
    long cap = (long)(2 * r + 1) * (2 * r + 1) * (2 * r + 1);
    int *off = (int *)malloc(sizeof(int) * 3 * cap);
    long noff = 0;
    for (int dz = -r; dz <= r; ++dz)
        for (int dy = -r; dy <= r; ++dy)
            for (int dx = -r; dx <= r; ++dx)
                if (dx * dx + dy * dy + dz * dz <= r * r) {
                    off[3 * noff] = dx;
                    off[3 * noff + 1] = dy;
                    off[3 * noff + 2] = dz;
                    ++noff;
                }
    long ns = *n_solid;
    long added = 0;
    while (added < max_spheres && (double)(ncell - ns) / (double)ncell > target_porosity) {
        int cx = (int)((sm_next(state) >> 32) % (uint64_t)nx);
        int cy = (int)((sm_next(state) >> 32) % (uint64_t)ny);
        int cz = (int)((sm_next(state) >> 32) % (uint64_t)nz);
        for (long k = 0; k < noff; ++k) {
            int x = ((cx + off[3 * k]) % nx + nx) % nx;
            int y = ((cy + off[3 * k + 1]) % ny + ny) % ny;
            int z = ((cz + off[3 * k + 2]) % nz + nz) % nz;
            long c = x + (long)nx * (y + (long)ny * z);
            if (!solid[c]) {
                solid[c] = 1;
                ++ns;
            }
        }
        ++added;
    }
    free(off);
    *n_solid = ns;
    return added;
}

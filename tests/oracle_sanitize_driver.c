/* Host sanitizer run of the stochastic-step oracle (test infrastructure).
 *
 * Built by tests/test_oracle_sanitize.py with gcc -fsanitize=address,undefined
 * together with oracle/fire_oracle.c (included below as one translation
 * unit).  Reads one batch from a binary input file, steps it with the
 * oracle's own entry points and writes the final states and counts, which the
 * test compares with the regular (unsanitized) oracle library.
 *
 * Input file (little-endian): int32 n_env, n_ign, T, n_threads, drop_mode,
 * drop_radius, flags (bit 0 actions, 1 per-env wind series, 2 per-cell wind
 * series, 3 static per-cell wind); int64 n_cells; uint64 seed, t0;
 * oracle_params; float veg[11]; uint32 unburnable_mask; oracle_env[n_env];
 * uint8 cls[n_cells]; float den[n_cells], elev[n_cells];
 * [float wind_cell[3][n_cells]]; int32 ign[n_ign][3];
 * [int32 actions[T][n_env]]; [float env_series[t0+T][n_env][3]];
 * [float cell_series[t0+T][3][n_cells]].
 * Output file: uint8 states[n_cells]; int32 counts[T][n_env]; float
 * exp_c and atan_c of 4096 fixed arguments.
 */
#include "../oracle/fire_oracle.c"

#include <stdio.h>

static void* read_block(FILE* f, size_t bytes)
{
    void* p = malloc(bytes ? bytes : 1);
    if (!p || fread(p, 1, bytes, f) != bytes) {
        fprintf(stderr, "short read (%zu bytes)\n", bytes);
        exit(2);
    }
    return p;
}

int main(int argc, char** argv)
{
    if (argc != 3) {
        fprintf(stderr, "usage: %s input output\n", argv[0]);
        return 2;
    }
    FILE* f = fopen(argv[1], "rb");
    if (!f) return 2;
    int32_t* hdr = (int32_t*)read_block(f, 7 * sizeof(int32_t));
    const int32_t n_env = hdr[0], n_ign = hdr[1], T = hdr[2], n_threads = hdr[3];
    const int32_t drop_mode = hdr[4], drop_radius = hdr[5], flags = hdr[6];
    int64_t* nc = (int64_t*)read_block(f, sizeof(int64_t));
    const int64_t n = nc[0];
    uint64_t* st = (uint64_t*)read_block(f, 2 * sizeof(uint64_t));
    const uint64_t seed = st[0], t0 = st[1];
    oracle_params* P = (oracle_params*)read_block(f, sizeof(oracle_params));
    float* veg = (float*)read_block(f, 11 * sizeof(float));
    uint32_t* mask = (uint32_t*)read_block(f, sizeof(uint32_t));
    oracle_env* envs = (oracle_env*)read_block(f, (size_t)n_env * sizeof(oracle_env));
    uint8_t* cls = (uint8_t*)read_block(f, (size_t)n);
    float* den = (float*)read_block(f, (size_t)n * sizeof(float));
    float* elev = (float*)read_block(f, (size_t)n * sizeof(float));
    float* wind_cell = (flags & 8) ? (float*)read_block(f, 3 * (size_t)n * sizeof(float)) : NULL;
    int32_t* ign = (int32_t*)read_block(f, 3 * (size_t)n_ign * sizeof(int32_t));
    int32_t* actions = (flags & 1) ? (int32_t*)read_block(f, (size_t)T * n_env * sizeof(int32_t)) : NULL;
    const size_t S = (size_t)(t0 + (uint64_t)T);
    float* env_series = (flags & 2) ? (float*)read_block(f, S * n_env * 3 * sizeof(float)) : NULL;
    float* cell_series = (flags & 4) ? (float*)read_block(f, S * 3 * (size_t)n * sizeof(float)) : NULL;
    fclose(f);

    float* g = (float*)malloc((size_t)n * sizeof(float));
    uint8_t* states = (uint8_t*)malloc((size_t)n);
    int32_t* counts = (int32_t*)malloc((size_t)T * n_env * sizeof(int32_t));
    oracle_fuel(n, cls, den, veg, g);
    if (oracle_init_states(n_env, envs, cls, mask[0], ign, n_ign, states) != 0) {
        fprintf(stderr, "bad ignition list\n");
        return 2;
    }
    oracle_run_ex(P, n_env, envs, g, elev, wind_cell, n, states, t0, T, actions, counts, seed, n_threads,
                  env_series, cell_series, drop_mode, drop_radius);

    float xs[4096], ye[4096], ya[4096];
    for (int i = 0; i < 4096; ++i) xs[i] = -100.0f + 0.05f * (float)i;
    oracle_exp_c_batch(xs, ye, 4096);
    oracle_atan_c_batch(xs, ya, 4096);

    FILE* o = fopen(argv[2], "wb");
    if (!o) return 2;
    fwrite(states, 1, (size_t)n, o);
    fwrite(counts, sizeof(int32_t), (size_t)T * n_env, o);
    fwrite(ye, sizeof(float), 4096, o);
    fwrite(ya, sizeof(float), 4096, o);
    fclose(o);
    free(hdr); free(nc); free(st); free(P); free(veg); free(mask); free(envs); free(cls); free(den);
    free(elev); free(wind_cell); free(ign); free(actions); free(env_series); free(cell_series);
    free(g); free(states); free(counts);
    return 0;
}

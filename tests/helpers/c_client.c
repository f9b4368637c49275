/* A plain C client of the transport library: it includes only mcx.h, links
 * only libmcx.so and owns only host memory.  It describes a two-slab,
 * two-group box, runs it on the asynchronous and the stack scheduler, checks
 * that both give the same integers, and writes the raw tally to a file
 * (argv[1]) for comparison with the CPU oracle.  Exit status 0 on success. */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "mcx.h"

#define CHECK(call)                                                                    \
    do {                                                                               \
        mcx_status s_ = (call);                                                        \
        if (s_ != MCX_OK) {                                                            \
            fprintf(stderr, "%s: %s (%s)\n", #call, mcx_status_str(s_), mcx_last_error(p)); \
            return 1;                                                                  \
        }                                                                              \
    } while (0)

int main(int argc, char **argv)
{
    if (argc < 2) return 2;
    static const double planes[3] = {0.0, 4.0, 10.0};
    static const int32_t slab_mat[2] = {0, 1};
    static const double sigma_t[4] = {1.0, 1.5, 0.6, 0.9};        /* [m][g] */
    static const double sigma_s[4] = {0.7, 1.2, 0.3, 0.5};
    static const double cdf[8] = {0.6, 1.0, 0.0, 1.0, 0.5, 1.0, 0.0, 1.0};   /* [m][g][g'] */
    static const double edges[6] = {0.0, 2.0, 4.0, 6.0, 8.0, 10.0};
    mcx_problem_desc d;
    memset(&d, 0, sizeof d);
    d.geometry = MCX_GEOM_BOX;
    for (int a = 0; a < 3; ++a) {
        d.box_lo[a] = 0.0;
        d.box_hi[a] = 10.0;
        d.src_pos[a] = 5.0;
        d.src_hi[a] = 10.0;
    }
    for (int f = 0; f < 6; ++f) d.bc[f] = MCX_BC_VACUUM;
    d.n_slabs = 2;
    d.slab_planes = planes;
    d.slab_mat = slab_mat;
    d.energy_mode = MCX_MG;
    d.n_mat = 2;
    d.n_grp = 2;
    d.sigma_t = sigma_t;
    d.sigma_s = sigma_s;
    d.transfer_cdf = cdf;
    d.src_kind = MCX_SRC_POINT;
    d.src_isotropic = 1;
    d.src_dir[0] = 1.0;
    d.tally_kind = MCX_TALLY_MESH;
    d.mesh_n[0] = d.mesh_n[1] = d.mesh_n[2] = 5;
    d.mesh_x = d.mesh_y = d.mesh_z = edges;
    d.tally_scale_log2 = 32;
    d.problem_id = 0;
    d.seed = 12345;
    d.n_histories = 50000;
    d.max_steps = 1000000;

    mcx_problem_t p = NULL;
    CHECK(mcx_create_problem(&d, 1, &p));
    int64_t n_bins = 0;
    CHECK(mcx_problem_info(p, 0, &n_bins, NULL, NULL, NULL));
    if (n_bins != 5 * 5 * 5 * 2) return 3;
    static int64_t a[250], b[250];
    mcx_run_opts o;
    memset(&o, 0, sizeof o);
    o.sched = MCX_SCHED_ASYNC;
    size_t ws = 0;
    CHECK(mcx_workspace_size(p, &o, &ws));
    CHECK(mcx_run(p, &o));
    CHECK(mcx_tallies(p, 0, a, n_bins, MCX_HOST));
    o.sched = MCX_SCHED_STACK;
    o.decomp = MCX_DECOMP_SPLIT;
    CHECK(mcx_run(p, &o));
    CHECK(mcx_tallies(p, 0, b, n_bins, MCX_HOST));
    if (memcmp(a, b, sizeof a) != 0) {
        fprintf(stderr, "schedulers disagree\n");
        return 4;
    }
    mcx_counters_t c;
    CHECK(mcx_counters(p, &c));
    /* a bad argument is an error status, not a crash */
    if (mcx_tallies(p, 0, a, n_bins + 1, MCX_HOST) != MCX_E_INVALID_ARG) return 5;
    mcx_destroy_problem(p);
    FILE *f = fopen(argv[1], "wb");
    if (!f) return 6;
    fwrite(a, sizeof(int64_t), (size_t)n_bins, f);
    fclose(f);
    printf("ok flights=%llu workspace=%zu\n", (unsigned long long)c.flights, ws);
    return 0;
}

/*
 * Memory and undefined-behaviour check of the CPU oracle (test infrastructure):
 * built by tests/test_oracle_sanitizers.py with AddressSanitizer and
 * UndefinedBehaviorSanitizer, it drives every entry point of the oracle on a
 * tiny object with every debug output enabled, over ordinary, axis-aligned,
 * face-grazing, inside-start and invalid rays (NaN, zero direction,
 * tmin > tmax, infinite origin).  Any sanitizer report aborts with a non-zero
 * exit status.
 */
#include "../oracle/lsnif_oracle.c"

#include <stdio.h>

static uint32_t lcg(uint32_t *s) { *s = *s * 1664525u + 1013904223u; return *s >> 8; }
static float unif(uint32_t *s) { return (float)lcg(s) / 16777216.0f; }

int main(void)
{
    uint32_t seed = 12345u;
    enum { V = 8, L = 2, F = 2, LOG2T = 6, H = 6, W1 = 16 };
    const int32_t R[L] = {5, 16};                      /* a hashed level and a face-aligned one */
    uint32_t occ[V * V * V / 32];
    for (int i = 0; i < V * V * V / 32; ++i) occ[i] = lcg(&seed) & lcg(&seed);
    static float tables[L << LOG2T][F];
    for (int i = 0; i < (L << LOG2T); ++i)
        for (int f = 0; f < F; ++f) tables[i][f] = unif(&seed) - 0.5f;
    const int32_t dims[4] = {H * L * F, W1, W1, 5 + 3 + 4};
    static float w0[W1 * H * L * F], w1[W1 * W1], w2[12 * W1];
    float *Ws[3] = {w0, w1, w2};
    const int sizes[3] = {W1 * H * L * F, W1 * W1, 12 * W1};
    for (int k = 0; k < 3; ++k)
        for (int i = 0; i < sizes[k]; ++i) Ws[k][i] = unif(&seed) - 0.5f;
    oracle_object ob;
    memset(&ob, 0, sizeof ob);
    for (int a = 0; a < 3; ++a) { ob.bmin[a] = -1.0f; ob.bmax[a] = 1.0f; }
    ob.V = V; ob.occ = occ; ob.L = L; ob.F = F; ob.log2_T = LOG2T; ob.R = R;
    ob.tables = &tables[0][0]; ob.H = H; ob.n_layers = 3; ob.dims = dims;
    ob.W = (const float *const *)Ws; ob.act = OR_LEAKY; ob.leaky_slope = 0.01f;
    ob.n_mat = 4; ob.has_albedo = 1;

    enum { N = 512 };
    static float rays[N][8];
    for (int i = 0; i < N; ++i) {
        for (int a = 0; a < 3; ++a) {
            rays[i][a] = 3.0f * (unif(&seed) - 0.5f);
            rays[i][3 + a] = unif(&seed) - 0.5f;
        }
        rays[i][6] = 0.0f;
        rays[i][7] = (i % 7 == 0) ? 1.5f : INFINITY;
        switch (i % 16) {
        case 1: rays[i][3] = 0.0f; rays[i][4] = 0.0f; rays[i][5] = 1.0f; break;     /* axis-aligned */
        case 2: rays[i][0] = 0.25f; rays[i][1] = -0.5f; rays[i][3] = 1.0f; rays[i][4] = 0.0f; rays[i][5] = 0.0f; break;   /* along grid planes */
        case 3: rays[i][0] = rays[i][1] = rays[i][2] = 0.1f; break;                 /* starts inside */
        case 4: rays[i][3] = NAN; break;                                           /* invalid */
        case 5: rays[i][3] = rays[i][4] = rays[i][5] = 0.0f; break;                 /* zero direction */
        case 6: rays[i][6] = 2.0f; rays[i][7] = 1.0f; break;                        /* tmin > tmax */
        case 7: rays[i][0] = INFINITY; break;                                      /* infinite origin */
        case 8: rays[i][0] = -1.0f; rays[i][1] = -1.0f; rays[i][2] = -2.0f; rays[i][3] = 0.0f; rays[i][4] = 0.0f; rays[i][5] = 1.0f; break;   /* along an edge of the box */
        default: break;
        }
    }
    static int32_t count[N], vox_ijk[N][H / 2][3], mat[N];
    static float tatb[N][2], vox_t[N][H / 2][2], points[N][H][3], weights[N][H][L][3], tt[N], nrm[N][3], alb[N][3];
    static int8_t vox_axis[N][H / 2][2];
    static uint32_t slots[N][H][L][8], hit[N];
    static double enc[N][H * L * F], out[N][12];
    oracle_outputs o = {&count[0], &tatb[0][0], &vox_ijk[0][0][0], &vox_t[0][0][0], &vox_axis[0][0][0],
                        &points[0][0][0], &slots[0][0][0][0], &weights[0][0][0][0], &enc[0][0], &out[0][0],
                        hit, tt, &nrm[0][0], mat, &alb[0][0]};
    if (oracle_query(&ob, &rays[0][0], N, &o) != 0) return 2;
    ob.grazing_recheck = 1;
    if (oracle_query(&ob, &rays[0][0], N, &o) != 0) return 3;

    /* two instances of the object: identity and a scaled, shifted copy */
    oracle_instance inst[2];
    memset(inst, 0, sizeof inst);
    inst[0].m[0] = inst[0].m[5] = inst[0].m[10] = 1.0f;
    inst[1].m[0] = inst[1].m[5] = inst[1].m[10] = 2.0f;
    inst[1].m[3] = 0.5f;
    static uint32_t counts[N + 1], pr[2 * N], pi[2 * N], wh[N];
    static int32_t winner[N];
    const int64_t np = oracle_broad_phase(&ob, inst, 2, &rays[0][0], N, counts, pr, pi, 2 * N);
    if (np < 0 || np > 2 * N) return 4;
    if (oracle_query_pairs(&ob, inst, 2, &rays[0][0], N, pr, pi, np, wh, tt, &nrm[0][0], mat, winner) != 0) return 5;
    static float next[N][8];
    static uint32_t parent[N];
    const int64_t nb = oracle_bounce(&rays[0][0], hit, tt, &nrm[0][0], N, 7u, 1u, 1e-4f, &next[0][0], parent);
    if (nb < 0 || nb > N) return 6;
    printf("ok: %lld pairs, %lld bounce rays\n", (long long)np, (long long)nb);
    return 0;
}

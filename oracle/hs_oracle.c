/*
 * hs_oracle.c -- plain FP64 CPU oracle for the hierarchy scan.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header or table with the
 * HIP implementation.
 *
 * Every routine is the plain definition written out, sequentially, in double
 * precision.  fp32 inputs are widened to double by the Python wrapper (an
 * exact conversion) before they reach these functions.
 *
 * Conventions (the readings of the paper that these routines fix):
 *   - matrices are 4x4, row-major, acting on column vectors;
 *   - a joint's local matrix is L = T(t) * R(q) * diag(s), q = (x, y, z, w);
 *   - the global ("model space") transform is G_j = G_parent(j) * L_j, the
 *     parent on the left as in the paper's Algorithms 1-4 (Sec. 2 and
 *     Sec. 3); the row-vector form of Eq. 1 is the transpose of this;
 *   - character-local parent indices, -1 marks a root, and every parent
 *     precedes its child (parent(j) < j), the ordering of Sec. 3.2.1.
 *
 * Return codes: 0 ok, 1 invalid argument, 2 topology violation.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stddef.h>
#include <string.h>

#define HSO_OK 0
#define HSO_EINVAL 1
#define HSO_ETOPO 2

/* C = A * B for 4x4 row-major doubles (C may not alias A or B). */
static void mat4_mul(const double *A, const double *B, double *C)
{
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) {
            double acc = 0.0;
            for (int k = 0; k < 4; ++k)
                acc += A[4 * r + k] * B[4 * k + c];
            C[4 * r + c] = acc;
        }
}

/* The textbook rotation matrix of the quaternion (x, y, z, w), used as given
 * (no renormalisation).  R[3*i+l] is row i, column l. */
static void quat_to_rot(const double *q, double *R)
{
    const double x = q[0], y = q[1], z = q[2], w = q[3];
    R[0] = 1.0 - 2.0 * (y * y + z * z);
    R[1] = 2.0 * (x * y - w * z);
    R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);
    R[4] = 1.0 - 2.0 * (x * x + z * z);
    R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);
    R[7] = 2.0 * (y * z + w * x);
    R[8] = 1.0 - 2.0 * (x * x + y * y);
}

/* Local matrix of one joint: [R(q) diag(s) | t ; 0 0 0 1]. */
static void trs_to_local(const double *q, const double *t, const double *s, double *L)
{
    double R[9];
    quat_to_rot(q, R);
    for (int i = 0; i < 3; ++i) {
        for (int l = 0; l < 3; ++l)
            L[4 * i + l] = R[3 * i + l] * (s ? s[l] : 1.0);
        L[4 * i + 3] = t[i];
    }
    L[12] = 0.0; L[13] = 0.0; L[14] = 0.0; L[15] = 1.0;
}

static int check_topology(int64_t C, const int64_t *offsets, const int32_t *parents)
{
    if (C < 0 || !offsets) return HSO_EINVAL;
    if (offsets[0] != 0) return HSO_EINVAL;
    for (int64_t c = 0; c < C; ++c) {
        if (offsets[c + 1] < offsets[c]) return HSO_EINVAL;
        const int64_t n = offsets[c + 1] - offsets[c];
        for (int64_t j = 0; j < n; ++j) {
            const int32_t p = parents[offsets[c] + j];
            if (p < -1 || (int64_t)p >= j) return HSO_ETOPO;
        }
    }
    return HSO_OK;
}

/* Local matrices of n joints from their TRS (scale may be NULL = unit). */
int hso_trs_to_local(int64_t n, const double *quat, const double *trans,
                     const double *scale, double *local)
{
    if (n < 0) return HSO_EINVAL;
    for (int64_t j = 0; j < n; ++j)
        trs_to_local(quat + 4 * j, trans + 3 * j, scale ? scale + 3 * j : NULL, local + 16 * j);
    return HSO_OK;
}

/*
 * Tree prefix product over given local matrices (Eq. 1 read with the
 * parent on the left, Sec. 3.1): for each character, in increasing joint
 * index, G_j = L_j at a root and G_j = G_parent(j) * L_j otherwise.
 */
int hso_scan_matrices(int64_t C, const int64_t *offsets, const int32_t *parents,
                      const double *local, double *global)
{
    int rc = check_topology(C, offsets, parents);
    if (rc) return rc;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t c = 0; c < C; ++c) {
        const int64_t base = offsets[c], n = offsets[c + 1] - offsets[c];
        for (int64_t j = 0; j < n; ++j) {
            const int32_t p = parents[base + j];
            const double *L = local + 16 * (base + j);
            double *G = global + 16 * (base + j);
            if (p < 0)
                memcpy(G, L, 16 * sizeof(double));
            else
                mat4_mul(global + 16 * (base + p), L, G);
        }
    }
    return HSO_OK;
}

/* Hierarchy-Scan (Sec. 1 step 2, Sec. 3): local TRS -> global matrices. */
int hso_forward(int64_t C, const int64_t *offsets, const int32_t *parents,
                const double *quat, const double *trans, const double *scale,
                double *global)
{
    int rc = check_topology(C, offsets, parents);
    if (rc) return rc;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t c = 0; c < C; ++c) {
        const int64_t base = offsets[c], n = offsets[c + 1] - offsets[c];
        for (int64_t j = 0; j < n; ++j) {
            const int64_t g = base + j;
            const int32_t p = parents[g];
            double L[16];
            trs_to_local(quat + 4 * g, trans + 3 * g, scale ? scale + 3 * g : NULL, L);
            if (p < 0)
                memcpy(global + 16 * g, L, sizeof L);
            else
                mat4_mul(global + 16 * (base + p), L, global + 16 * g);
        }
    }
    return HSO_OK;
}

/* Bind MeshPose (Sec. 1 step 3): skin_j = global_j * inv_bind_j, 4x4. */
int hso_skin(int64_t n, const double *global, const double *inv_bind, double *skin)
{
    if (n < 0) return HSO_EINVAL;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j)
        mat4_mul(global + 16 * j, inv_bind + 16 * j, skin + 16 * j);
    return HSO_OK;
}

/*
 * Root-to-joint path length lambda_j = sum over the path nodes k of
 * |A_parent(k) t_k| (A of a root's parent is the identity): the length of
 * the polyline of joint origins from the root to j, used to scale the
 * translation tolerance.
 */
int hso_path_length(int64_t C, const int64_t *offsets, const int32_t *parents,
                    const double *global, const double *trans, double *lambda)
{
    int rc = check_topology(C, offsets, parents);
    if (rc) return rc;
    for (int64_t c = 0; c < C; ++c) {
        const int64_t base = offsets[c], n = offsets[c + 1] - offsets[c];
        for (int64_t j = 0; j < n; ++j) {
            const int64_t g = base + j;
            const int32_t p = parents[g];
            const double *t = trans + 3 * g;
            double v[3];
            if (p < 0) {
                v[0] = t[0]; v[1] = t[1]; v[2] = t[2];
                lambda[g] = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
            } else {
                const double *A = global + 16 * (base + p);
                for (int i = 0; i < 3; ++i)
                    v[i] = A[4 * i + 0] * t[0] + A[4 * i + 1] * t[1] + A[4 * i + 2] * t[2];
                lambda[g] = lambda[base + p] + sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
            }
        }
    }
    return HSO_OK;
}

/* ---------------------------------------------------------------------- */
/* Simulation step (Sec. 1 step 1): sample two looping clips and blend.     */
/* The paper leaves this step to existing practice; the reading fixed here  */
/* is: per clip, keys k0 = floor(fps*tau) mod K and k1 = k0+1 mod K, a      */
/* normalised lerp of the key quaternions (taking the shorter arc) and a    */
/* plain lerp of translations; then the two clips blended the same way with */
/* the character's weight.                                                   */
/* ---------------------------------------------------------------------- */

/* Sign decision for the shorter arc.  Both this oracle and the GPU kernel
 * decide it from the same fp64 sum of the four exact fp32*fp32 products,
 * added in the order x, y, z, w, so the two sides never disagree. */
static double key_dot_sign_source(const float *a, const float *b)
{
    double d = (double)a[0] * (double)b[0];
    d = d + (double)a[1] * (double)b[1];
    d = d + (double)a[2] * (double)b[2];
    d = d + (double)a[3] * (double)b[3];
    return d;
}

static void nlerp_d(const double *a, const double *b, double sigma, double alpha, double *out)
{
    double n2 = 0.0;
    for (int k = 0; k < 4; ++k) {
        out[k] = (1.0 - alpha) * a[k] + alpha * sigma * b[k];
        n2 += out[k] * out[k];
    }
    const double inv = 1.0 / sqrt(n2);
    for (int k = 0; k < 4; ++k) out[k] *= inv;
}

/*
 * key_quat [clips][keys][J][4], key_trans [clips][keys][J][3] (fp32 values
 * widened by the caller only for the arithmetic below: the keys themselves
 * stay fp32 so the arc decision can be taken exactly).  Per character c:
 * clip_a[c], clip_b[c], time[c] (seconds), weight[c].  Joint j of character
 * c samples joint j of the clip, so n_c <= J is required.
 */
int hso_pose_sample(int64_t C, const int64_t *offsets,
                    int32_t num_clips, int32_t num_keys, int32_t J, float fps,
                    const float *key_quat, const float *key_trans,
                    const int32_t *clip_a, const int32_t *clip_b,
                    const float *time, const float *weight,
                    double *quat_out, double *trans_out)
{
    if (C < 0 || num_clips <= 0 || num_keys <= 0 || J <= 0) return HSO_EINVAL;
    for (int64_t c = 0; c < C; ++c) {
        if (offsets[c + 1] - offsets[c] > J) return HSO_EINVAL;
        if (clip_a[c] < 0 || clip_a[c] >= num_clips || clip_b[c] < 0 || clip_b[c] >= num_clips)
            return HSO_EINVAL;
    }
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < C; ++c) {
        /* frame position f = fps * tau in FP64 from the fp32 inputs */
        const double f = (double)fps * (double)time[c];
        const double fl = floor(f);
        const double alpha = f - fl;
        int64_t k0 = (int64_t)fl % num_keys;
        if (k0 < 0) k0 += num_keys;
        const int64_t k1 = (k0 + 1) % num_keys;
        const double w = (double)weight[c];
        const int32_t clips[2] = {clip_a[c], clip_b[c]};
        const int64_t base = offsets[c], n = offsets[c + 1] - offsets[c];
        for (int64_t j = 0; j < n; ++j) {
            double qc[2][4], tc[2][3];
            for (int s = 0; s < 2; ++s) {
                const int64_t r0 = ((int64_t)clips[s] * num_keys + k0) * J + j;
                const int64_t r1 = ((int64_t)clips[s] * num_keys + k1) * J + j;
                const float *qa = key_quat + 4 * r0, *qb = key_quat + 4 * r1;
                const double sigma = key_dot_sign_source(qa, qb) < 0.0 ? -1.0 : 1.0;
                double a[4], b[4];
                for (int k = 0; k < 4; ++k) { a[k] = qa[k]; b[k] = qb[k]; }
                nlerp_d(a, b, sigma, alpha, qc[s]);
                for (int i = 0; i < 3; ++i)
                    tc[s][i] = (1.0 - alpha) * (double)key_trans[3 * r0 + i] + alpha * (double)key_trans[3 * r1 + i];
            }
            double d = 0.0;
            for (int k = 0; k < 4; ++k) d += qc[0][k] * qc[1][k];
            const double sigma = d < 0.0 ? -1.0 : 1.0;
            nlerp_d(qc[0], qc[1], sigma, w, quat_out + 4 * (base + j));
            for (int i = 0; i < 3; ++i)
                trans_out[3 * (base + j) + i] = (1.0 - w) * tc[0][i] + w * tc[1][i];
        }
    }
    return HSO_OK;
}

/* ---------------------------------------------------------------------- */
/* Adjoint of the hierarchy scan (reverse mode of G_j = G_p * L_j).         */
/* For a product C = A*B the adjoints are  Abar += Cbar * B^T  and          */
/* Bbar += A^T * Cbar.  Children have larger indices than their parents, so */
/* a sweep from the last joint to the first sees every child's complete     */
/* adjoint before adding it into the parent.                                 */
/* ---------------------------------------------------------------------- */
int hso_backward(int64_t C, const int64_t *offsets, const int32_t *parents,
                 const double *quat, const double *trans, const double *scale,
                 const double *grad_global, double *grad_quat, double *grad_trans,
                 double *grad_scale /* nullable */, double *work /* [N,16] adjoints */,
                 double *global /* [N,16] */)
{
    int rc = hso_forward(C, offsets, parents, quat, trans, scale, global);
    if (rc) return rc;
    const int64_t N = offsets[C];
    memcpy(work, grad_global, (size_t)N * 16 * sizeof(double));
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t c = 0; c < C; ++c) {
        const int64_t base = offsets[c], n = offsets[c + 1] - offsets[c];
        for (int64_t j = n - 1; j >= 0; --j) {
            const int64_t g = base + j;
            const int32_t p = parents[g];
            const double *s = scale ? scale + 3 * g : NULL;
            double L[16], Lt[16], Gpt[16], Lbar[16];
            trs_to_local(quat + 4 * g, trans + 3 * g, s, L);
            const double *Gbar = work + 16 * g;
            if (p >= 0) {
                /* parent adjoint += Gbar_j * L_j^T */
                double acc[16];
                for (int r = 0; r < 4; ++r)
                    for (int k = 0; k < 4; ++k) Lt[4 * r + k] = L[4 * k + r];
                mat4_mul(Gbar, Lt, acc);
                double *Pbar = work + 16 * (base + p);
                for (int k = 0; k < 16; ++k) Pbar[k] += acc[k];
                /* Lbar_j = G_p^T * Gbar_j */
                const double *Gp = global + 16 * (base + p);
                for (int r = 0; r < 4; ++r)
                    for (int k = 0; k < 4; ++k) Gpt[4 * r + k] = Gp[4 * k + r];
                mat4_mul(Gpt, Gbar, Lbar);
            } else {
                memcpy(Lbar, Gbar, sizeof Lbar);
            }
            /* L = [R diag(s) | t]: split Lbar into the rotation-scale block and t */
            double R[9];
            quat_to_rot(quat + 4 * g, R);
            double Rbar[9];
            for (int i = 0; i < 3; ++i)
                for (int l = 0; l < 3; ++l)
                    Rbar[3 * i + l] = Lbar[4 * i + l] * (s ? s[l] : 1.0);
            for (int i = 0; i < 3; ++i) grad_trans[3 * g + i] = Lbar[4 * i + 3];
            if (grad_scale)
                for (int l = 0; l < 3; ++l) {
                    double a = 0.0;
                    for (int i = 0; i < 3; ++i) a += Lbar[4 * i + l] * R[3 * i + l];
                    grad_scale[3 * g + l] = a;
                }
            /* d R_il / d q_k of the polynomial in quat_to_rot */
            const double x = quat[4 * g + 0], y = quat[4 * g + 1], z = quat[4 * g + 2], w = quat[4 * g + 3];
            const double dR[4][9] = {
                /* d/dx */ {0, 2 * y, 2 * z, 2 * y, -4 * x, -2 * w, 2 * z, 2 * w, -4 * x},
                /* d/dy */ {-4 * y, 2 * x, 2 * w, 2 * x, 0, 2 * z, -2 * w, 2 * z, -4 * y},
                /* d/dz */ {-4 * z, -2 * w, 2 * x, 2 * w, -4 * z, 2 * y, 2 * x, 2 * y, 0},
                /* d/dw */ {0, -2 * z, 2 * y, 2 * z, 0, -2 * x, -2 * y, 2 * x, 0},
            };
            for (int k = 0; k < 4; ++k) {
                double a = 0.0;
                for (int e = 0; e < 9; ++e) a += Rbar[e] * dR[k][e];
                grad_quat[4 * g + k] = a;
            }
        }
    }
    return HSO_OK;
}

/* Thread count for the parallel loops over characters (n >= 1); returns the
 * count now in effect.  Changes no arithmetic: characters are independent. */
int hso_set_threads(int n)
{
    if (n >= 1) omp_set_num_threads(n);
    return omp_get_max_threads();
}

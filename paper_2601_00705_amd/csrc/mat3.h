// mat3.h -- small double-precision 3x3 helpers shared by the merging and
// the seed initialisation: a symmetric eigen-decomposition and the unit
// quaternion of a rotation matrix.
#pragma once

namespace gsr {

// symmetric 3x3 eigen-decomposition S = V diag(lam) V^T by cyclic Jacobi
// rotations (S is overwritten)
__device__ __forceinline__ void eig3(double (&S)[3][3], double (&V)[3][3], double (&lam)[3])
{
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) V[r][c] = r == c ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 30; ++sweep) {
        const double off = S[0][1] * S[0][1] + S[0][2] * S[0][2] + S[1][2] * S[1][2];
        const double on = S[0][0] * S[0][0] + S[1][1] * S[1][1] + S[2][2] * S[2][2];
        if (!(off > 1e-32 * on)) break;
#pragma unroll
        for (int p = 0; p < 2; ++p) {
#pragma unroll
            for (int q = p + 1; q < 3; ++q) {
                if (S[p][q] == 0.0) continue;
                const double th = (S[q][q] - S[p][p]) / (2.0 * S[p][q]);
                const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                // S <- J^T S J, V <- V J, J the rotation in the (p, q) plane
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const double skp = S[k][p], skq = S[k][q];
                    S[k][p] = c * skp - s * skq;
                    S[k][q] = s * skp + c * skq;
                }
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const double spk = S[p][k], sqk = S[q][k];
                    S[p][k] = c * spk - s * sqk;
                    S[q][k] = s * spk + c * sqk;
                }
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const double vkp = V[k][p], vkq = V[k][q];
                    V[k][p] = c * vkp - s * vkq;
                    V[k][q] = s * vkp + c * vkq;
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) lam[k] = S[k][k];
}

// a unit quaternion (w, x, y, z) of the rotation matrix R (largest of the
// four squared components first, for accuracy)
__device__ __forceinline__ void rot_quat(const double (&R)[3][3], double (&q)[4])
{
    const double tr = R[0][0] + R[1][1] + R[2][2];
    if (tr >= R[0][0] && tr >= R[1][1] && tr >= R[2][2]) {
        const double s = 2.0 * sqrt(1.0 + tr);
        q[0] = 0.25 * s;
        q[1] = (R[2][1] - R[1][2]) / s;
        q[2] = (R[0][2] - R[2][0]) / s;
        q[3] = (R[1][0] - R[0][1]) / s;
    } else if (R[0][0] >= R[1][1] && R[0][0] >= R[2][2]) {
        const double s = 2.0 * sqrt(1.0 + R[0][0] - R[1][1] - R[2][2]);
        q[0] = (R[2][1] - R[1][2]) / s;
        q[1] = 0.25 * s;
        q[2] = (R[0][1] + R[1][0]) / s;
        q[3] = (R[0][2] + R[2][0]) / s;
    } else if (R[1][1] >= R[2][2]) {
        const double s = 2.0 * sqrt(1.0 + R[1][1] - R[0][0] - R[2][2]);
        q[0] = (R[0][2] - R[2][0]) / s;
        q[1] = (R[0][1] + R[1][0]) / s;
        q[2] = 0.25 * s;
        q[3] = (R[1][2] + R[2][1]) / s;
    } else {
        const double s = 2.0 * sqrt(1.0 + R[2][2] - R[0][0] - R[1][1]);
        q[0] = (R[1][0] - R[0][1]) / s;
        q[1] = (R[0][2] + R[2][0]) / s;
        q[2] = (R[1][2] + R[2][1]) / s;
        q[3] = 0.25 * s;
    }
}

}  // namespace gsr

// ag_camera.hip -- depth images by ray casting against primitive obstacles.
//
// One block renders a 64 x 4 pixel tile of one vehicle's camera: each
// wavefront owns one 64-pixel row segment (one coalesced 256-byte store).
// The block first places the camera (vehicle pose composed with the mount)
// and moves the camera origin into every obstacle's frame once, keeping the
// per-obstacle constants (rotation, origin in the obstacle frame, size, type)
// in LDS.  Each lane then rotates its ray into each obstacle frame and runs
// the slab / quadratic intersection of that obstacle's type; every lane of
// the block tests the same obstacle at the same time, so there is no
// divergence between shapes.  Depth is the distance along the optical axis
// of the first entry (exit when the camera is inside a solid), clipped to
// the camera's maximum depth.
#include <hip/hip_runtime.h>

#include "ag.h"
#include "ag_internal.h"

namespace ag {

constexpr int CAM_TX = 64, CAM_TY = 4;
constexpr int OBST_LDS = 16;      // floats per obstacle in LDS
constexpr int kMaxObstacles = 256;

__device__ __forceinline__ void quat_rot(float w, float x, float y, float z, float* R) {
    R[0] = 1.0f - 2.0f * (y * y + z * z); R[1] = 2.0f * (x * y - w * z); R[2] = 2.0f * (x * z + w * y);
    R[3] = 2.0f * (x * y + w * z); R[4] = 1.0f - 2.0f * (x * x + z * z); R[5] = 2.0f * (y * z - w * x);
    R[6] = 2.0f * (x * z - w * y); R[7] = 2.0f * (y * z + w * x); R[8] = 1.0f - 2.0f * (x * x + y * y);
}

// entry if ahead, else exit if ahead (origin inside), else miss
__device__ __forceinline__ float first_positive(float tn, float tf, bool hit) {
    const float t = tn > 0.0f ? tn : (tf > 0.0f ? tf : INFINITY);
    return hit ? t : INFINITY;
}

__global__ __launch_bounds__(256) void k_depth(CameraArgs a) {
    __shared__ float ob[kMaxObstacles * OBST_LDS];
    __shared__ float cam[12];                     // R_wc (9) and origin (3)
    const long long v = a.first + blockIdx.y;    // vehicle
    const int tiles_x = (a.W + CAM_TX - 1) / CAM_TX;
    const int tx = blockIdx.x % tiles_x, ty = blockIdx.x / tiles_x;
    const int tid = threadIdx.x;

    if (tid == 0) {
        float Rb[9], Rm[9];
        quat_rot(a.state[6 * a.ld + v], a.state[7 * a.ld + v], a.state[8 * a.ld + v], a.state[9 * a.ld + v], Rb);
        quat_rot(a.mount_q[0], a.mount_q[1], a.mount_q[2], a.mount_q[3], Rm);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                cam[3 * i + j] = Rb[3 * i] * Rm[j] + Rb[3 * i + 1] * Rm[3 + j] + Rb[3 * i + 2] * Rm[6 + j];
        for (int i = 0; i < 3; ++i)
            cam[9 + i] = a.state[i * a.ld + v] + Rb[3 * i] * a.mount_p[0] + Rb[3 * i + 1] * a.mount_p[1] +
                         Rb[3 * i + 2] * a.mount_p[2];
    }
    __syncthreads();
    for (int k = tid; k < a.n_obs; k += blockDim.x) {
        const long long oi = v * a.n_obs + k;
        const float* sh = a.shapes + k * 8;
        float R[9];
        quat_rot(a.obst[3 * a.obst_ld + oi], a.obst[4 * a.obst_ld + oi], a.obst[5 * a.obst_ld + oi],
                 a.obst[6 * a.obst_ld + oi], R);
        const float px = cam[9] - a.obst[oi], py = cam[10] - a.obst[a.obst_ld + oi],
                    pz = cam[11] - a.obst[2 * a.obst_ld + oi];
        float* o = ob + k * OBST_LDS;
        for (int j = 0; j < 9; ++j) o[j] = R[j];
        o[9] = R[0] * px + R[3] * py + R[6] * pz;    // camera origin in the obstacle frame: R^T (p - c)
        o[10] = R[1] * px + R[4] * py + R[7] * pz;
        o[11] = R[2] * px + R[5] * py + R[8] * pz;
        o[12] = sh[0];
        o[13] = sh[1];
        o[14] = sh[2];
        o[15] = sh[3];
    }
    __syncthreads();

    const int u = tx * CAM_TX + (tid & 63);
    const int row = ty * CAM_TY + (tid >> 6);
    if (u >= a.W || row >= a.H) return;
    // ray in the camera frame (x forward, y left, z up), then in the world frame
    const float dcx = 1.0f, dcy = -((float)u + 0.5f - 0.5f * (float)a.W) * a.inv_f,
                dcz = -((float)row + 0.5f - 0.5f * (float)a.H) * a.inv_f;
    const float in = __builtin_amdgcn_rsqf(dcx * dcx + dcy * dcy + dcz * dcz);
    const float cx = dcx * in, cy = dcy * in, cz = dcz * in;
    const float dx = cam[0] * cx + cam[1] * cy + cam[2] * cz;
    const float dy = cam[3] * cx + cam[4] * cy + cam[5] * cz;
    const float dz = cam[6] * cx + cam[7] * cy + cam[8] * cz;
    float t = INFINITY;
    if (a.has_floor && dz < 0.0f && cam[11] > a.floor_z) {
        const float tp = (a.floor_z - cam[11]) / dz;
        t = tp > 0.0f ? tp : t;
    }
    for (int k = 0; k < a.n_obs; ++k) {
        const float* o = ob + k * OBST_LDS;
        const float lx = o[0] * dx + o[3] * dy + o[6] * dz;     // ray direction in the obstacle frame
        const float ly = o[1] * dx + o[4] * dy + o[7] * dz;
        const float lz = o[2] * dx + o[5] * dy + o[8] * dz;
        const float ox = o[9], oy = o[10], oz = o[11];
        const int typ = (int)o[12];
        float tk;
        if (typ == 0) {                                        // box, slab method
            const float ix = 1.0f / lx, iy = 1.0f / ly, iz = 1.0f / lz;
            const float ax = (-o[13] - ox) * ix, bx = (o[13] - ox) * ix;
            const float ay = (-o[14] - oy) * iy, by = (o[14] - oy) * iy;
            const float az = (-o[15] - oz) * iz, bz = (o[15] - oz) * iz;
            const float tn = fmaxf(fmaxf(fminf(ax, bx), fminf(ay, by)), fminf(az, bz));
            const float tf = fminf(fminf(fmaxf(ax, bx), fmaxf(ay, by)), fmaxf(az, bz));
            tk = first_positive(tn, tf, tn <= tf);
        } else if (typ == 1) {                                 // sphere
            const float b = ox * lx + oy * ly + oz * lz;
            const float c = ox * ox + oy * oy + oz * oz - o[13] * o[13];
            const float disc = b * b - c;
            const float s = sqrtf(fmaxf(disc, 0.0f));
            tk = first_positive(-b - s, -b + s, disc >= 0.0f);
        } else {                                               // capped cylinder along local z
            const float A = lx * lx + ly * ly;
            const float b = ox * lx + oy * ly;
            const float c = ox * ox + oy * oy - o[13] * o[13];
            const float disc = b * b - A * c;
            const float s = sqrtf(fmaxf(disc, 0.0f));
            float tsi, tso;
            bool side_ok;
            if (A > 0.0f) {
                const float iA = 1.0f / A;
                tsi = (-b - s) * iA;
                tso = (-b + s) * iA;
                side_ok = disc >= 0.0f;
            } else {
                tsi = c <= 0.0f ? -INFINITY : INFINITY;
                tso = c <= 0.0f ? INFINITY : -INFINITY;
                side_ok = c <= 0.0f;
            }
            float tzi, tzo;
            if (lz != 0.0f) {
                const float iz = 1.0f / lz;
                const float t1 = (-o[14] - oz) * iz, t2 = (o[14] - oz) * iz;
                tzi = fminf(t1, t2);
                tzo = fmaxf(t1, t2);
            } else {
                const bool within = fabsf(oz) <= o[14];
                tzi = within ? -INFINITY : INFINITY;
                tzo = within ? INFINITY : -INFINITY;
            }
            const float tn = fmaxf(tsi, tzi), tf = fminf(tso, tzo);
            tk = first_positive(tn, tf, side_ok && tn <= tf);
        }
        t = fminf(t, tk);
    }
    const float depth = t * cx;
    a.depth[((long long)blockIdx.y * a.H + row) * a.W + u] = (depth <= a.max_depth) ? depth : a.max_depth;
}

const void* depth_kernel() { return reinterpret_cast<const void*>(&k_depth); }

}  // namespace ag

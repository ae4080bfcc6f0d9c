// ag_camera.hip -- depth images by ray casting against primitive obstacles.
//
// One block renders a 64 x 4 pixel tile of one vehicle's camera: each
// wavefront owns one 64-pixel row segment (one coalesced 256-byte store).
// The block first places the camera (vehicle pose composed with the mount)
// and moves the camera origin into every obstacle's frame once, keeping the
// per-obstacle constants (rotation, origin in the obstacle frame, size, type)
// in LDS, and lists the obstacles whose bounding sphere meets the cone of the
// tile's rays within max_depth (the others cannot change a pixel of it).  Each lane then rotates its ray into each obstacle frame and runs
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

// Hardware reciprocal and square root (1 ulp): rcp(+-0) = +-inf as for 1/x,
// which the slab tests rely on for directions parallel to a face.
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float sqrt1(float x) { return __builtin_amdgcn_sqrtf(x); }

// entry if ahead, else exit if ahead (origin inside), else miss
__device__ __forceinline__ float first_positive(float tn, float tf, bool hit) {
    const float t = tn > 0.0f ? tn : (tf > 0.0f ? tf : INFINITY);
    return hit ? t : INFINITY;
}

// Camera-frame ray direction (not normalised) through the centre of pixel (u, row).
__device__ __forceinline__ void pixel_dir(const CameraArgs& a, float u, float row, float& y, float& z) {
    y = -(u + 0.5f - 0.5f * (float)a.W) * a.inv_f;
    z = -(row + 0.5f - 0.5f * (float)a.H) * a.inv_f;
}

__global__ __launch_bounds__(256) void k_depth(CameraArgs a) {
    __shared__ float ob[kMaxObstacles * OBST_LDS];
    __shared__ float cam[12];                     // R_wc (9) and origin (3)
    __shared__ float cone[5];                     // tile axis (world), cos and sin of its half-angle
    __shared__ float cx_min;                      // smallest optical-axis cosine of the tile's rays
    __shared__ int keepf[kMaxObstacles];
    __shared__ int keep[kMaxObstacles];
    __shared__ int nkeep;
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
        // the tile's rays lie in the cone over its corner rays: axis through
        // the tile centre, half-angle the largest corner angle (FP64, once per block)
        const float u0 = (float)(tx * CAM_TX), r0 = (float)(ty * CAM_TY);
        const float u1 = (float)(min(tx * CAM_TX + CAM_TX, a.W) - 1), r1 = (float)(min(ty * CAM_TY + CAM_TY, a.H) - 1);
        float yc, zc;
        pixel_dir(a, 0.5f * (u0 + u1), 0.5f * (r0 + r1), yc, zc);
        const double nc = sqrt(1.0 + (double)yc * yc + (double)zc * zc);
        const double ax = 1.0 / nc, ay = yc / nc, az = zc / nc;
        double cmin = 1.0, xmin = 1.0;
        const float cu[4] = {u0, u1, u0, u1}, cr[4] = {r0, r0, r1, r1};
        for (int c = 0; c < 4; ++c) {
            float y, z;
            pixel_dir(a, cu[c], cr[c], y, z);
            const double n = sqrt(1.0 + (double)y * y + (double)z * z);
            cmin = fmin(cmin, (ax + ay * y + az * z) / n);
            xmin = fmin(xmin, 1.0 / n);
        }
        for (int i = 0; i < 3; ++i)
            cone[i] = (float)(cam[3 * i] * ax + cam[3 * i + 1] * ay + cam[3 * i + 2] * az);
        cone[3] = (float)cmin;
        cone[4] = (float)sqrt(fmax(0.0, 1.0 - cmin * cmin));
        cx_min = (float)xmin;
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
        // Culling: the obstacle lies in its bounding sphere (centre, radius br);
        // skip it when that sphere misses the tile's cone, or when even its
        // nearest point is past max_depth along every ray of the tile (such a
        // hit would be clipped to max_depth anyway).  FP64 with a margin, so
        // that no obstacle a ray could hit is skipped.
        const int typ = (int)sh[0];
        const double h1 = sh[1], h2 = sh[2], h3 = sh[3];
        const double br = (typ == 0 ? sqrt(h1 * h1 + h2 * h2 + h3 * h3) : typ == 1 ? h1 : sqrt(h1 * h1 + h2 * h2)) *
                              (1.0 + 1e-4) + 1e-5;
        const double vx = -(double)px, vy = -(double)py, vz = -(double)pz;   // centre - camera
        const double dist = sqrt(vx * vx + vy * vy + vz * vz);
        int kp = 1;
        if (dist > br) {
            const double sb = br / dist, cb = sqrt(fmax(0.0, 1.0 - sb * sb));
            const double cth = (cone[0] * vx + cone[1] * vy + cone[2] * vz) / dist;
            const double cab = (double)cone[3] * cb - (double)cone[4] * sb;   // cos(alpha + beta)
            kp = cth >= cab - 1e-7;
            if ((dist - br) * (double)cx_min > (double)a.max_depth * (1.0 + 1e-4)) kp = 0;
        }
        keepf[k] = kp;
    }
    __syncthreads();
    if (tid == 0) {
        int m = 0;
        for (int k = 0; k < a.n_obs; ++k)
            if (keepf[k]) keep[m++] = k;
        nkeep = m;
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
    const int nk = nkeep;
    for (int kk = 0; kk < nk; ++kk) {
        const float* o = ob + keep[kk] * OBST_LDS;
        const float lx = o[0] * dx + o[3] * dy + o[6] * dz;     // ray direction in the obstacle frame
        const float ly = o[1] * dx + o[4] * dy + o[7] * dz;
        const float lz = o[2] * dx + o[5] * dy + o[8] * dz;
        const float ox = o[9], oy = o[10], oz = o[11];
        const int typ = (int)o[12];
        float tk;
        if (typ == 0) {                                        // box, slab method
            const float ix = rcp(lx), iy = rcp(ly), iz = rcp(lz);
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
            const float s = sqrt1(fmaxf(disc, 0.0f));
            tk = first_positive(-b - s, -b + s, disc >= 0.0f);
        } else {                                               // capped cylinder along local z
            const float A = lx * lx + ly * ly;
            const float b = ox * lx + oy * ly;
            const float c = ox * ox + oy * oy - o[13] * o[13];
            const float disc = b * b - A * c;
            const float s = sqrt1(fmaxf(disc, 0.0f));
            float tsi, tso;
            bool side_ok;
            if (A > 0.0f) {
                const float iA = rcp(A);
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
                const float iz = rcp(lz);
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

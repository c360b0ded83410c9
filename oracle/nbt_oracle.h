/*
 * nbt_oracle.h -- interface of the CPU oracle (test infrastructure only).
 * The definitions and conventions are documented in nbt_oracle.c.
 */
#ifndef NBT_ORACLE_H
#define NBT_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORACLE_MISS = 0, ORACLE_HIT = 1, ORACLE_END = 2, ORACLE_EXIT = 3, ORACLE_INVALID = 4 };
enum { ORACLE_OCCUPIED = 1, ORACLE_FREE = 2, ORACLE_UNKNOWN = 3 };

typedef struct {
    const float* P;          /* [nz][ny][nx] occupancy probabilities, x fastest */
    int32_t nx, ny, nz;
    float voxel;             /* s_Vox in metres */
    float origin[3];         /* world position of the min corner of voxel (0,0,0) */
    float occ_threshold;     /* Occupied if P > occ_threshold */
    float free_threshold;    /* Free if P < free_threshold; Unknown otherwise */
} oracle_map;

typedef struct {
    int32_t width, height;   /* endpoint grid on the far plane */
    float tan_half_h, tan_half_v;
    float range;             /* d_Cam */
} oracle_camera;

typedef struct {
    uint32_t steps;          /* voxels visited (N_O) */
    int32_t stop_lin;        /* linear index of the last visited voxel, -1 if none */
    int32_t reason;          /* ORACLE_MISS / HIT / END / EXIT / INVALID */
    uint64_t hash;           /* FNV-1a-64 over the visited linear indices (4 LE bytes each) */
    double gain;             /* g_R */
} oracle_ray;

uint64_t oracle_fnv1a_bytes(const uint8_t* bytes, int64_t n);
void oracle_cast_ray(const oracle_map* m, const oracle_camera* cam, const float* pose,
                     int i, int j, int32_t* path, int path_cap, oracle_ray* out);
void oracle_trace_rays(const oracle_map* m, const oracle_camera* cam, const float* poses,
                       int64_t n_poses, uint32_t* steps, int32_t* stop_lin, int32_t* reason,
                       uint64_t* hash, double* gain);
void oracle_eval_viewpoints(const oracle_map* m, const oracle_camera* cam, const float* poses,
                            int64_t n_poses, float* ig_out, uint64_t* steps_out);
int oracle_eval_trajectories(const oracle_map* m, const oracle_camera* cam, const float* poses,
                             int64_t n_traj, int64_t poses_per_traj, float* ig_union,
                             uint32_t* counts, uint64_t* visits);
int oracle_insert_scans(const oracle_map* m, const oracle_camera* cam, const float* poses,
                        const float* depth, int64_t n_scans, float l_hit, float l_miss,
                        float l_min, float l_max, float* logodds);

#ifdef __cplusplus
}
#endif

#endif

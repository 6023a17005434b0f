// rc_index.hip -- static node table of a forest share (Sec. 2.1): the internal
// nodes of the trees above the leaves, built level by level from the leaves
// in space-filling-curve order.  A level-l internal node is the common
// level-l ancestor of a run of consecutive leaves deeper than l.
#include "rc_host.h"
#include "rc_internal.h"

namespace rc {
namespace {

// Tree of leaf i from the tree offsets.
__device__ inline int tree_of(const int64_t* tb, int ntrees, int64_t i) {
    int k = 0;
    while (k + 1 < ntrees && i >= tb[k + 1]) k++;
    return k;
}

__device__ inline bool tree_start(const int64_t* tb, int ntrees, int64_t i) {
    for (int k = 0; k <= ntrees; k++)
        if (tb[k] == i) return true;
    return false;
}

// status[0]: error flags, status[1]: maximum level, status[2]: leaf levels (bit mask)
__global__ void k_validate(int64_t n, const uint8_t* level, const uint32_t* x, const uint32_t* y, const uint32_t* z,
                           const int64_t* tb, int ntrees, int maxallowed, int flat, int* status) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (level[i] > maxallowed) atomicOr(&status[0], 8);
    int l = level[i];
    if (l > QMAX) {
        atomicOr(&status[0], 1);
        return;
    }
    uint32_t len = 1u << (QMAX - l);
    if ((flat && z[i] != 0) || (x[i] & (len - 1)) || (y[i] & (len - 1)) || (z[i] & (len - 1)) || x[i] + len > (1u << QMAX) ||
        y[i] + len > (1u << QMAX) || z[i] + len > (1u << QMAX)) {
        atomicOr(&status[0], 2);
        return;
    }
    atomicMax(&status[1], l);
    atomicOr(&status[2], 1 << l);
    if (i > 0 && !tree_start(tb, ntrees, i)) {
        int lp = level[i - 1];
        if (lp > QMAX) return;
        uint64_t kp = morton(x[i - 1], y[i - 1], z[i - 1]);
        uint64_t span = (uint64_t)1 << (3 * (QMAX - lp));
        if (kp + span > morton(x[i], y[i], z[i])) atomicOr(&status[0], 4);
    }
}

__global__ void k_fill_i32(int64_t n, int32_t* p, int32_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

struct OpenItem {
    int64_t val;
};

// leaf i opens the level-l node that contains it iff it is the first leaf of it
struct OpenSrc {
    const uint8_t* level;
    const uint32_t *x, *y, *z;
    int l;
    const int64_t* tb;
    int ntrees;
    __device__ OpenItem operator()(int64_t i) const {
        OpenItem it;
        it.val = 0;
        if (level[i] <= l) return it;
        if (i == 0 || level[i - 1] <= l || tree_start(tb, ntrees, i)) {
            it.val = 1;
            return it;
        }
        int sh = QMAX - l;
        it.val = ((x[i - 1] >> sh) != (x[i] >> sh) || (y[i - 1] >> sh) != (y[i] >> sh) ||
                  (z[i - 1] >> sh) != (z[i] >> sh))
                     ? 1
                     : 0;
        return it;
    }
};

struct OpenDst {
    const uint8_t* level;
    const uint32_t *x, *y, *z;
    int l;
    int64_t base, cap;
    int32_t* cur;  // per leaf: its internal node at the previous level
    int32_t* child;
    uint8_t* nlevel;
    uint32_t *nx, *ny, *nz;
    uint8_t* ntree;
    const int64_t* tb;
    int ntrees;
    int32_t* roots;
    int64_t* count;
    __device__ void operator()(int64_t i, int64_t pre, const OpenItem& it) const {
        if (level[i] <= l) return;
        int64_t node = base + pre + it.val - 1;  // node of level l holding leaf i
        int sh = QMAX - l;
        if (it.val && node < cap) {
            int tr = tree_of(tb, ntrees, i);
            ntree[node] = (uint8_t)tr;
            if (l == 0) roots[tr] = (int32_t)node;
            nlevel[node] = (uint8_t)l;
            nx[node] = (x[i] >> sh) << sh;
            ny[node] = (y[i] >> sh) << sh;
            nz[node] = (z[i] >> sh) << sh;
            if (l > 0) {
                int32_t parent = cur[i];
                int d = ((x[i] >> sh) & 1) | (((y[i] >> sh) & 1) << 1) | (((z[i] >> sh) & 1) << 2);
                if (parent >= 0 && parent < cap) child[(int64_t)parent * 8 + d] = (int32_t)node;
            }
        }
        if (level[i] == l + 1 && node < cap) {
            int s1 = QMAX - l - 1;
            int d = ((x[i] >> s1) & 1) | (((y[i] >> s1) & 1) << 1) | (((z[i] >> s1) & 1) << 2);
            child[node * 8 + d] = (int32_t)(-2 - i);
        }
        cur[i] = (int32_t)(node < cap ? node : -1);
    }
    __device__ void total(int64_t t) const { *count = t; }
};

}  // namespace
}  // namespace rc

using namespace rc;

extern "C" rc_status rc_forest_index(const rc_forest* f, rc_index* ix, void* ws, size_t ws_bytes, void* stream) {
    rc_status s = check_forest(f);
    if (s != RC_OK) return s;
    if (!ix) return RC_EINVAL;
    if (!ws || ws_bytes < rc_workspace_bytes(f, nullptr, 1, nullptr)) return RC_EWORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    int64_t N = f->nleaves;
    int nt = f->ntrees;
    char* w = (char*)ws;
    int* status = (int*)(w + IX_STATUS);
    int64_t* dcount = (int64_t*)(w + IX_COUNT);
    int64_t* dtb = (int64_t*)(w + IX_TREES);
    int32_t* droots = (int32_t*)(w + IX_ROOTS);
    int32_t* cur = (int32_t*)(w + IX_CUR);
    int64_t* partial = (int64_t*)(w + IX_CUR + align_up((size_t)N * 4));

    int64_t htb[RC_MAXTREES + 1];
    int32_t hroots[RC_MAXTREES];
    for (int k = 0; k <= nt; k++) htb[k] = f->tree_begin ? f->tree_begin[k] : (k == 0 ? 0 : N);
    for (int k = 0; k < nt; k++) hroots[k] = htb[k + 1] > htb[k] ? (int32_t)(-2 - htb[k]) : RC_ABSENT;
    int maxallowed = RC_QMAXLEVEL;
    if (is_shell(f)) {
        double L = 0.0;
        RC_HIP(hipMemcpyAsync(&L, f->geom_table + 2, sizeof(double), hipMemcpyDeviceToHost, st));
        RC_HIP(hipStreamSynchronize(st));
        if (!(L >= 0.0 && L <= RC_QMAXLEVEL && L == (double)(int)L)) return RC_EINVAL;
        maxallowed = (int)L;
    }
    RC_HIP(hipMemcpyAsync(dtb, htb, sizeof(int64_t) * (nt + 1), hipMemcpyHostToDevice, st));
    RC_HIP(hipMemcpyAsync(droots, hroots, sizeof(int32_t) * nt, hipMemcpyHostToDevice, st));
    RC_HIP(hipMemsetAsync(status, 0, 64, st));
    unsigned nb = (unsigned)((N + 255) / 256);
    hipLaunchKernelGGL(k_validate, dim3(nb), dim3(256), 0, st, N, f->level, f->x, f->y, f->z, (const int64_t*)dtb, nt,
                       maxallowed, is_surface(f) ? 1 : 0, status);
    RC_HIP(hipGetLastError());
    int hs[3];
    RC_HIP(hipMemcpyAsync(hs, status, sizeof(hs), hipMemcpyDeviceToHost, st));
    RC_HIP(hipStreamSynchronize(st));
    if (hs[0] != 0) return RC_EFOREST;
    int maxlevel = hs[1];
    for (int k = 0; k < nt; k++)
        if (maxlevel == 0 && htb[k + 1] - htb[k] > 1) return RC_EFOREST;
    ix->maxlevel = maxlevel;
    ix->leaf_levels = hs[2];
    ix->ntrees = nt;

    // all capacity-guarded: a first pass with too little room still counts
    bool have = ix->child && ix->level && ix->x && ix->y && ix->z && ix->tree && ix->cap_internal > 0;
    int64_t cap = have ? ix->cap_internal : 0;
    if (have) {
        unsigned g = (unsigned)((cap * 8 + 255) / 256);
        hipLaunchKernelGGL(k_fill_i32, dim3(g), dim3(256), 0, st, cap * 8, ix->child, (int32_t)RC_ABSENT);
        RC_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_fill_i32, dim3(nb), dim3(256), 0, st, N, cur, (int32_t)-1);
    RC_HIP(hipGetLastError());
    int64_t base = 0;
    for (int l = 0; l < maxlevel; l++) {
        ix->level_begin[l] = base;
        OpenSrc src{f->level, f->x, f->y, f->z, l, (const int64_t*)dtb, nt};
        OpenDst dst{f->level, f->x,  f->y,  f->z,  l,     base,     cap,      cur,    ix->child,
                    ix->level, ix->x, ix->y, ix->z, ix->tree, (const int64_t*)dtb, nt, droots, dcount};
        RC_HIP(launch_scan<int64_t>(N, src, dst, partial, st));
        int64_t cnt = 0;
        RC_HIP(hipMemcpyAsync(&cnt, dcount, sizeof(cnt), hipMemcpyDeviceToHost, st));
        RC_HIP(hipStreamSynchronize(st));
        base += cnt;
    }
    for (int l = maxlevel; l < RC_QMAXLEVEL + 2; l++) ix->level_begin[l] = base;
    ix->ninternal = base;
    if (base > cap) return RC_ECAPACITY;
    RC_HIP(hipMemcpyAsync(hroots, droots, sizeof(int32_t) * nt, hipMemcpyDeviceToHost, st));
    RC_HIP(hipStreamSynchronize(st));
    for (int k = 0; k < RC_MAXTREES; k++) ix->roots[k] = k < nt ? hroots[k] : RC_ABSENT;
    ix->root = hroots[0];
    return RC_OK;
}

"""FP64 oracle of vertex skinning -- TEST INFRASTRUCTURE ONLY.

The step after the paper's pipeline (Sec. 3 names skinning among the GPU
stages; the experiment of Sec. 4 skins meshes of 1000-3000 faces): each
vertex of a character's mesh is moved by a weighted blend of the skin
matrices S_j = G_j B_j^-1 of up to four joints.

* ``linear_blend`` -- linear blend skinning: p' = sum_i w_i S_{j_i} [p, 1],
  the weights used as given.
* ``dual_quaternion`` -- dual quaternion skinning (Kavan, Collins, Zara and
  O'Sullivan, "Geometric skinning with approximate dual quaternion
  blending", ACM TOG 2008): each rigid S_j becomes a unit dual quaternion
  (q_r, q_d) with q_d = 1/2 (t, 0) q_r; the influences are summed with
  weights w_i times the sign of q_r,i . q_r,0 (slot 0 is the pivot), the
  sum is divided by the norm of its real part, and the resulting rigid
  transform is applied to p.  The rotation block of S is read as a rotation
  (scale is not part of the method); its quaternion comes from SciPy.

Batch layout (as the library's hs_mesh): character c owns output rows
vertex_offsets[c] .. vertex_offsets[c+1]-1; its k-th vertex uses mesh row
mesh_first[c] + k of positions [M,3], joints [M,4] (character-local joint
ids) and weights [M,4]; S rows are offsets[c] + joint id.

Parity status: pinned by closed forms in tests/test_oracle_vertex_skin.py
(translations, common-axis rotations, the twisting joint, the antipodal
sign rule, rigidity).
"""
import numpy as np
from scipy.spatial.transform import Rotation


def _gather(offsets, skin, vertex_offsets, mesh_first, joints):
    """Per output vertex: its mesh row and the four skin matrices it uses."""
    C = len(offsets) - 1
    counts = np.diff(np.asarray(vertex_offsets, np.int64))
    rows = np.concatenate([np.arange(mesh_first[c], mesh_first[c] + counts[c]) for c in range(C)]) \
        if C else np.zeros(0, np.int64)
    char = np.repeat(np.arange(C), counts)
    jid = np.asarray(joints, np.int64)[rows]
    S = np.asarray(skin, np.float64)[np.asarray(offsets, np.int64)[char][:, None] + jid]  # [V,4,4,4]
    return rows, S


def linear_blend(offsets, skin, vertex_offsets, mesh_first, positions, joints, weights):
    rows, S = _gather(offsets, skin, vertex_offsets, mesh_first, joints)
    p = np.asarray(positions, np.float64)[rows]
    w = np.asarray(weights, np.float64)[rows]
    ph = np.concatenate([p, np.ones((p.shape[0], 1))], axis=1)
    moved = np.einsum("vkab,vb->vka", S[:, :, :3, :], ph)  # each influence's S_j [p, 1]
    return np.einsum("vk,vka->va", w, moved)


def _qmul(a, b):
    """Hamilton product of quaternions stored (x, y, z, w), batched."""
    ax, ay, az, aw = np.moveaxis(a, -1, 0)
    bx, by, bz, bw = np.moveaxis(b, -1, 0)
    return np.stack([aw * bx + ax * bw + ay * bz - az * by,
                     aw * by - ax * bz + ay * bw + az * bx,
                     aw * bz + ax * by - ay * bx + az * bw,
                     aw * bw - ax * bx - ay * by - az * bz], axis=-1)


def _conj(q):
    return q * np.array([-1.0, -1.0, -1.0, 1.0])


def dual_quaternions(S):
    """Unit dual quaternion (q_r, q_d) of each rigid 4x4 transform."""
    S = np.asarray(S, np.float64)
    shape = S.shape[:-2]
    flat = S.reshape(-1, 4, 4)
    qr = Rotation.from_matrix(flat[:, :3, :3]).as_quat()  # (x, y, z, w), unit
    t = np.concatenate([flat[:, :3, 3], np.zeros((flat.shape[0], 1))], axis=1)
    qd = 0.5 * _qmul(t, qr)
    return qr.reshape(shape + (4,)), qd.reshape(shape + (4,))


def dual_quaternion(offsets, skin, vertex_offsets, mesh_first, positions, joints, weights):
    rows, S = _gather(offsets, skin, vertex_offsets, mesh_first, joints)
    p = np.asarray(positions, np.float64)[rows]
    w = np.asarray(weights, np.float64)[rows]
    qr, qd = dual_quaternions(S)  # [V,4,4] each
    sign = np.where(np.einsum("vka,va->vk", qr, qr[:, 0, :]) < 0.0, -1.0, 1.0)
    ws = w * sign
    br = np.einsum("vk,vka->va", ws, qr)
    bd = np.einsum("vk,vka->va", ws, qd)
    n = np.linalg.norm(br, axis=1, keepdims=True)
    br, bd = br / n, bd / n
    # rotate p by br, then translate by 2 vec(bd conj(br))
    pq = np.concatenate([p, np.zeros((p.shape[0], 1))], axis=1)
    rotated = _qmul(_qmul(br, pq), _conj(br))[:, :3]
    trans = 2.0 * _qmul(bd, _conj(br))[:, :3]
    return rotated + trans


def skin_vertices(method, *args):
    """method 0: linear blend; 1: dual quaternion."""
    return (linear_blend if method == 0 else dual_quaternion)(*args)

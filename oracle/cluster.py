"""Cross-DM candidate clustering (beyond the paper: its search phase, section 2.2,
defers to the single-pulse work it cites, which groups the detections of one pulse
across neighbouring trials and starts).

TEST INFRASTRUCTURE, like the rest of `oracle/`.

Definition (friends of friends): two candidates of the same beam are linked iff their
trial indices differ by at most dm_radius and their starts by at most t_radius. A
cluster is a connected component of the links. Each cluster reports:
  peak     its member with the highest S/N; among equal S/N the smallest (dm_idx, t)
  members  the number of members
  dm_lo, dm_hi, t_lo, t_hi   the smallest and largest trial and start of the members
Clusters are listed in (beam, peak dm_idx, peak t) order.
"""


def cluster(cands, dm_radius: int, t_radius: int, beams=None):
    """cands: list of (dm_idx, t, width, snr) tuples; beams: optional beam id per
    candidate (0 for all by default). Returns a list of dicts in output order. Every pair
    is tested (quadratic): for small lists only."""
    n = len(cands)
    beams = [0] * n if beams is None else list(beams)
    parent = list(range(n))

    def find(i):
        while parent[i] != i:
            parent[i] = parent[parent[i]]
            i = parent[i]
        return i

    for i in range(n):
        for j in range(i + 1, n):
            if (beams[i] == beams[j] and abs(cands[i][0] - cands[j][0]) <= dm_radius
                    and abs(cands[i][1] - cands[j][1]) <= t_radius):
                ri, rj = find(i), find(j)
                if ri != rj:
                    parent[max(ri, rj)] = min(ri, rj)
    groups = {}
    for i in range(n):
        groups.setdefault(find(i), []).append(i)
    out = []
    for members in groups.values():
        best = min(members, key=lambda i: (-cands[i][3], cands[i][0], cands[i][1]))
        out.append(dict(beam=beams[best], peak=cands[best], members=len(members),
                        dm_lo=min(cands[i][0] for i in members), dm_hi=max(cands[i][0] for i in members),
                        t_lo=min(cands[i][1] for i in members), t_hi=max(cands[i][1] for i in members)))
    out.sort(key=lambda c: (c["beam"], c["peak"][0], c["peak"][1]))
    return out

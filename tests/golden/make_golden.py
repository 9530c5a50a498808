"""Writes soup256_oracle.txt: a digest of the oracle's K-pass render of the
256-triangle workload (calls only the oracle and the seeded input generator)."""
import hashlib
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle      # noqa: E402
import scenegen    # noqa: E402


def digest():
    w = scenegen.workload("soup256")
    img, ids = oracle.OracleScene(w.scene, use_bvh=False).render(
        w.camera, w.width, w.height, w.passes, w.lambda_eye, w.lambda_dir, nthreads=1)
    return {
        "images_sha256": hashlib.sha256(img.tobytes()).hexdigest(),
        "ids_sha256": hashlib.sha256(ids.tobytes()).hexdigest(),
        "hit_pixels_pass0": int((ids[0] >= 0).sum()),
        "changed_pixels_pass5": int((img[5] != img[4]).any(-1).sum()),
    }


if __name__ == "__main__":
    d = digest()
    with open(os.path.join(HERE, "soup256_oracle.txt"), "w") as f:
        for k, v in d.items():
            f.write(f"{k} {v}\n")
    print(d)

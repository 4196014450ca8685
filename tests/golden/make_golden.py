"""Write the closed-form golden fixtures (no oracle or HIP code involved)."""
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def grid64_hist():
    return [min(k + 1, 127 - k, 64) for k in range(127)]


if __name__ == "__main__":
    with open(os.path.join(HERE, "grid64_levels_hist.txt"), "w") as f:
        f.write("# BFS from vertex 0 on the 64x64 4-neighbour grid: vertices per level\n")
        f.write("# level k holds min(k+1, 127-k, 64) vertices (Manhattan distance r+c)\n")
        for k, v in enumerate(grid64_hist()):
            f.write(f"{k} {v}\n")

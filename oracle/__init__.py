"""Plain FP64 CPU oracle for L-JSDE / RL-JSDE. Test infrastructure only."""
